"""Python binding of the MI355X fusion library (libfuseflow.so, C ABI in include/fuseflow.h).

Argument marshalling only: every step of the fusion path runs in the HIP kernels of the
library.  PyTorch provides device memory and streams.  If the shared library is missing
this module raises at import time — there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, List, Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfuseflow.so")

FF_OK, FF_ERR_INVALID_ARG, FF_ERR_OOM, FF_ERR_BUSY, FF_ERR_HIP, FF_ERR_NOT_FOUND = range(6)
FF_NO_MF, FF_NO_DC, FF_NO_SA, FF_CONF_EQ3 = 1, 2, 4, 8
FF_DEV_OK, FF_DEV_OVERFLOW, FF_DEV_ERROR = 0, 1, 2
PAD = 0xFFFFFFFF


class FuseFlowError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {_lib.ff_status_string(status).decode()} ({status})")


# ----------------------------------------------------------------------------- C structs

class ff_camera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("world_to_cam", ctypes.c_float * 12)]


class ff_view(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_void_p), ("conf", ctypes.c_void_p), ("rgb", ctypes.c_void_p)]


class ff_params(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_float), ("k_views", ctypes.c_int32),
                ("sigma", ctypes.c_float), ("coarse_res", ctypes.c_int32),
                ("max_level", ctypes.c_int32), ("target_per_cell", ctypes.c_int32),
                ("level_override", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class ff_output(ctypes.Structure):
    _fields_ = [("xyz", ctypes.c_void_p), ("weight", ctypes.c_void_p), ("rgb", ctypes.c_void_p),
                ("n_members", ctypes.c_void_p), ("reps", ctypes.c_void_p),
                ("keys", ctypes.c_void_p), ("member_offsets", ctypes.c_void_p),
                ("member_ids", ctypes.c_void_p), ("capacity", ctypes.c_uint32),
                ("member_capacity", ctypes.c_uint32), ("count", ctypes.c_void_p),
                ("status", ctypes.c_void_p), ("info", ctypes.c_void_p)]


class ff_frame(ctypes.Structure):
    _fields_ = [("n_cams", ctypes.c_int32), ("cams", ctypes.POINTER(ff_camera)),
                ("views", ctypes.POINTER(ff_view))]


class ff_tuning(ctypes.Structure):
    _fields_ = [("radix_bits", ctypes.c_int32), ("sort_items", ctypes.c_int32),
                ("hist_tiles", ctypes.c_int32), ("cell_groups", ctypes.c_int32),
                ("use_graph", ctypes.c_int32)]


class ff_trace(ctypes.Structure):
    _fields_ = [("total_ms", ctypes.c_double * 32), ("launches", ctypes.c_uint64 * 32),
                ("calls", ctypes.c_uint64)]


class ff_probe(ctypes.Structure):
    _fields_ = [("slot", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("launches", ctypes.c_uint64), ("frames", ctypes.c_uint64),
                ("pixels", ctypes.c_uint64), ("total_ms", ctypes.c_double)]


class ff_conf_params(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_float), ("beta", ctypes.c_float),
                ("gamma", ctypes.c_float), ("delta", ctypes.c_float)]


class ff_emc_params(ctypes.Structure):
    _fields_ = [("c_occ", ctypes.c_float), ("stride", ctypes.c_int32)]


class ff_server_config(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("lanes", ctypes.c_int32),
                ("max_batch_frames", ctypes.c_int32), ("max_cameras", ctypes.c_int32),
                ("max_pending", ctypes.c_int32), ("plain", ctypes.c_int32),
                ("autotune", ctypes.c_int32)]


class ff_stats(ctypes.Structure):
    _fields_ = [("frames", ctypes.c_uint64), ("pixels", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("first_arrival_s", ctypes.c_double),
                ("last_done_s", ctypes.c_double), ("p50_ms", ctypes.c_double),
                ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
                ("max_ms", ctypes.c_double), ("px_per_s", ctypes.c_double),
                ("mean_batch_frames", ctypes.c_double), ("hbm_used_bytes", ctypes.c_uint64),
                ("hbm_peak_bytes", ctypes.c_uint64)]


# ----------------------------------------------------------------------------- library

EXPORTS = {
    "ff_version": (ctypes.c_char_p, []),
    "ff_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "ff_params_default": (None, [ctypes.POINTER(ff_params)]),
    "ff_context_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                         ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32]),
    "ff_context_destroy": (None, [ctypes.c_void_p]),
    "ff_workspace_bytes": (ctypes.c_uint64, [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32]),
    "ff_fuse": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ff_camera),
                               ctypes.POINTER(ff_view), ctypes.POINTER(ff_params),
                               ctypes.POINTER(ff_output), ctypes.c_void_p]),
    "ff_fuse_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ff_frame),
                                     ctypes.POINTER(ff_params), ctypes.POINTER(ff_output),
                                     ctypes.c_void_p]),
    "ff_get_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ff_tuning)]),
    "ff_set_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ff_tuning)]),
    "ff_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ff_frame),
                                   ctypes.POINTER(ff_params), ctypes.POINTER(ff_output),
                                   ctypes.c_void_p, ctypes.POINTER(ff_tuning)]),
    "ff_tuning_lookup": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ff_frame),
                                        ctypes.POINTER(ff_params), ctypes.POINTER(ff_tuning),
                                        ctypes.POINTER(ctypes.c_int32)]),
    "ff_tuning_export": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_uint64,
                                        ctypes.POINTER(ctypes.c_uint64)]),
    "ff_tuning_import": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p,
                                        ctypes.POINTER(ctypes.c_int32)]),
    "ff_trace_enable": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "ff_trace_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ff_trace)]),
    "ff_trace_slot_name": (ctypes.c_char_p, [ctypes.c_int32]),
    "ff_conf_params_default": (None, [ctypes.POINTER(ff_conf_params)]),
    "ff_confidence": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ff_camera),
                                     ctypes.POINTER(ff_view), ctypes.POINTER(ctypes.c_void_p),
                                     ctypes.POINTER(ff_conf_params), ctypes.c_void_p]),
    "ff_emc_params_default": (None, [ctypes.POINTER(ff_emc_params)]),
    "ff_emc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ff_camera),
                              ctypes.POINTER(ff_view), ctypes.c_void_p, ctypes.c_void_p,
                              ctypes.c_uint32, ctypes.POINTER(ff_emc_params), ctypes.c_void_p,
                              ctypes.c_void_p]),
    "ff_emc_noalloc": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ff_camera),
                                      ctypes.POINTER(ff_view), ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_uint32, ctypes.POINTER(ff_emc_params),
                                      ctypes.c_void_p, ctypes.c_void_p]),
    "ff_probe_enable": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "ff_probe_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ff_probe)]),
    "ff_server_config_default": (None, [ctypes.POINTER(ff_server_config)]),
    "ff_server_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                        ctypes.POINTER(ff_server_config)]),
    "ff_server_destroy": (None, [ctypes.c_void_p]),
    "ff_server_max_pixels": (ctypes.c_uint64, [ctypes.c_void_p]),
    "ff_server_now": (ctypes.c_double, [ctypes.c_void_p]),
    "ff_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ff_frame),
                                        ctypes.POINTER(ff_params), ctypes.POINTER(ff_output),
                                        ctypes.c_double, ctypes.c_void_p,
                                        ctypes.POINTER(ctypes.c_uint64)]),
    "ff_server_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64,
                                      ctypes.POINTER(ctypes.c_int32)]),
    "ff_server_wait": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "ff_server_drain": (ctypes.c_int, [ctypes.c_void_p]),
    "ff_server_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ff_stats)]),
    "ff_server_reset_stats": (ctypes.c_int, [ctypes.c_void_p]),
    "ff_server_reserve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32,
                                         ctypes.c_int32]),
    "ff_server_latencies": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64,
                                           ctypes.POINTER(ctypes.c_int32),
                                           ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_uint64)]),
    "ff_server_probe_enable": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "ff_server_probe_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ff_probe)]),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2602_01035_amd/build.py "
                          "first")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def lib():
    return _lib


def version() -> str:
    return _lib.ff_version().decode()


# ----------------------------------------------------------------------------- helpers

class Params:
    """ff_params with the library defaults; keyword overrides."""

    def __init__(self, **kw):
        p = ff_params()
        _lib.ff_params_default(ctypes.byref(p))
        for k, v in kw.items():
            if not hasattr(p, k):
                raise TypeError(f"unknown parameter {k!r}")
            setattr(p, k, v)
        self.c = p

    def __getattr__(self, k):
        return getattr(self.__dict__["c"], k)


def _check(status: int, where: str):
    if status != FF_OK:
        raise FuseFlowError(status, where)


def _probe_dict(p: ff_probe) -> Dict:
    return dict(slot=int(p.slot), launches=int(p.launches), frames=int(p.frames),
                pixels=int(p.pixels), total_ms=float(p.total_ms),
                mean_ms=float(p.total_ms) / p.launches if p.launches else 0.0)


def _camera(cam) -> ff_camera:
    c = ff_camera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    T = [float(v) for row in cam.world_to_cam for v in row]
    if len(T) != 12:
        raise ValueError("world_to_cam must be 3x4")
    for i, v in enumerate(T):
        c.world_to_cam[i] = v
    return c


def _torch():
    import torch
    return torch


def _check_image(t, H, W, dtype, name, channels=None):
    torch = _torch()
    shape = (H, W) if channels is None else (H, W, channels)
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError(f"{name} must be a ROCm device tensor")
    if t.dtype != dtype or tuple(t.shape) != shape or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} tensor of shape {shape}")


def _stream_ptr(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Output:
    """Device output buffers of one frame (torch tensors) and the ff_output view of them."""

    def __init__(self, capacity: int, member_capacity: int = 0, rgb: bool = False,
                 members: bool = False, device=None):
        torch = _torch()
        dev = device or torch.device("cuda", torch.cuda.current_device())
        cap = max(1, int(capacity))
        self.capacity = cap
        self.xyz = torch.empty((cap, 3), dtype=torch.float32, device=dev)
        self.weight = torch.empty(cap, dtype=torch.float32, device=dev)
        self.rgb = torch.empty((cap, 3), dtype=torch.uint8, device=dev) if rgb else None
        self.n_members = torch.empty(cap, dtype=torch.int32, device=dev)
        self.reps = torch.empty((cap, 3), dtype=torch.int32, device=dev)
        self.keys = torch.empty(cap, dtype=torch.int64, device=dev)
        self.member_offsets = torch.empty(cap + 1, dtype=torch.int32, device=dev) if members else None
        mcap = max(1, int(member_capacity)) if members else 0
        self.member_capacity = mcap
        self.member_ids = torch.empty(mcap, dtype=torch.int32, device=dev) if members else None
        self.count = torch.zeros(1, dtype=torch.int32, device=dev)
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        self.info = torch.zeros(4, dtype=torch.int32, device=dev)

    def c(self) -> ff_output:
        o = ff_output()
        ptr = lambda t: t.data_ptr() if t is not None else None
        o.xyz, o.weight, o.rgb = ptr(self.xyz), ptr(self.weight), ptr(self.rgb)
        o.n_members, o.reps, o.keys = ptr(self.n_members), ptr(self.reps), ptr(self.keys)
        o.member_offsets, o.member_ids = ptr(self.member_offsets), ptr(self.member_ids)
        o.capacity, o.member_capacity = self.capacity, self.member_capacity
        o.count, o.status, o.info = ptr(self.count), ptr(self.status), ptr(self.info)
        return o

    def result(self) -> Dict:
        """Synchronise and return the fused cloud as NumPy arrays (cells in key order)."""
        import numpy as np
        _torch().cuda.synchronize()
        S = int(self.count.item())
        st = int(self.status.item())
        n = min(S, self.capacity)
        u32 = lambda t: t.cpu().numpy().view(np.uint32)
        out = dict(count=S, status=st, xyz=self.xyz[:n].cpu().numpy(),
                   weight=self.weight[:n].cpu().numpy(),
                   rgb=self.rgb[:n].cpu().numpy() if self.rgb is not None else None,
                   n_members=u32(self.n_members[:n]), reps=u32(self.reps[:n]),
                   keys=self.keys[:n].cpu().numpy().view(np.uint64),
                   info=u32(self.info))
        if self.member_offsets is not None:
            M = int(out["info"][0])
            out["member_offsets"] = u32(self.member_offsets[:n + 1])
            out["member_ids"] = u32(self.member_ids[:min(M, self.member_capacity)])
        return out


class Context:
    """A device workspace for batches of up to max_frames frames / max_pixels pixels."""

    def __init__(self, max_pixels: int, max_cameras: int = 64, max_frames: int = 1,
                 device: Optional[int] = None):
        torch = _torch()
        if device is None:
            device = torch.cuda.current_device()
        self.device = device
        h = ctypes.c_void_p()
        _check(_lib.ff_context_create(ctypes.byref(h), device, int(max_pixels),
                                      int(max_cameras), int(max_frames)), "ff_context_create")
        self.h = h
        self.max_pixels, self.max_cameras, self.max_frames = max_pixels, max_cameras, max_frames

    def close(self):
        if getattr(self, "h", None):
            _lib.ff_context_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- tuning
    def tuning(self) -> Dict:
        t = ff_tuning()
        _check(_lib.ff_get_tuning(self.h, ctypes.byref(t)), "ff_get_tuning")
        return {k: getattr(t, k) for k, _ in ff_tuning._fields_}

    def set_tuning(self, **kw):
        t = ff_tuning()
        _check(_lib.ff_get_tuning(self.h, ctypes.byref(t)), "ff_get_tuning")
        for k, v in kw.items():
            setattr(t, k, int(v))
        _check(_lib.ff_set_tuning(self.h, ctypes.byref(t)), "ff_set_tuning")

    # -- kernel timing
    def trace(self, on: bool = True):
        _check(_lib.ff_trace_enable(self.h, int(on)), "ff_trace_enable")

    def trace_read(self) -> Dict:
        t = ff_trace()
        _check(_lib.ff_trace_read(self.h, ctypes.byref(t)), "ff_trace_read")
        out = {}
        for s in range(32):
            if t.launches[s]:
                out[_lib.ff_trace_slot_name(s).decode()] = dict(
                    slot=s, total_ms=t.total_ms[s], launches=int(t.launches[s]),
                    mean_ms=t.total_ms[s] / t.launches[s])
        return dict(calls=int(t.calls), kernels=out)

    def probe(self, slot: int):
        """Time trace slot `slot` in every later call (-1: off); resets the totals."""
        _check(_lib.ff_probe_enable(self.h, int(slot)), "ff_probe_enable")

    def probe_read(self) -> Dict:
        p = ff_probe()
        _check(_lib.ff_probe_read(self.h, ctypes.byref(p)), "ff_probe_read")
        return _probe_dict(p)

    # -- marshalling
    @staticmethod
    def _views(cams, depth, conf, rgb):
        """ff_camera / ff_view arrays; conf may be None (FF_CONF_EQ3 computes it)."""
        torch = _torch()
        n = len(cams)
        if conf is None:
            conf = [None] * n
        if len(depth) != n or len(conf) != n or (rgb is not None and len(rgb) != n):
            raise ValueError("one depth, confidence (and rgb) image per camera")
        ccams = (ff_camera * n)()
        views = (ff_view * n)()
        for k, cam in enumerate(cams):
            ccams[k] = _camera(cam)
            H, W = int(cam.height), int(cam.width)
            _check_image(depth[k], H, W, torch.float32, f"depth[{k}]")
            views[k].depth = depth[k].data_ptr()
            if conf[k] is not None:
                _check_image(conf[k], H, W, torch.float32, f"conf[{k}]")
                views[k].conf = conf[k].data_ptr()
            if rgb is not None:
                _check_image(rgb[k], H, W, torch.uint8, f"rgb[{k}]", channels=3)
                views[k].rgb = rgb[k].data_ptr()
        return ccams, views

    def fuse(self, cams, depth: Sequence, conf: Sequence, rgb: Optional[Sequence] = None,
             params: Optional[Params] = None, out: Optional[Output] = None, stream=None,
             members: bool = False) -> Output:
        """One frame through the per-step kernels (ff_fuse). Asynchronous on `stream`."""
        ccams, views = self._views(cams, depth, conf, rgb)
        P = sum(int(c.width) * int(c.height) for c in cams)
        if out is None:
            out = Output(P, P, rgb=rgb is not None, members=members)
        prm = (params or Params()).c
        o = out.c()
        _check(_lib.ff_fuse(self.h, len(cams), ccams, views, ctypes.byref(prm), ctypes.byref(o),
                            _stream_ptr(stream)), "ff_fuse")
        return out

    def _frames(self, frames):
        keep, cf = [], (ff_frame * len(frames))()
        for f, fr in enumerate(frames):
            ccams, views = self._views(fr["cams"], fr["depth"], fr.get("conf"), fr.get("rgb"))
            keep.append((ccams, views))
            cf[f].n_cams = len(fr["cams"])
            cf[f].cams = ctypes.cast(ccams, ctypes.POINTER(ff_camera))
            cf[f].views = ctypes.cast(views, ctypes.POINTER(ff_view))
        return cf, keep

    def fuse_batch(self, frames: List[Dict], params: Optional[Params] = None,
                   outs: Optional[List[Output]] = None, stream=None,
                   members: bool = False) -> List[Output]:
        """Several frames in one batched call (ff_fuse_batch, replayed from a cached
        graph).  Each frame is a dict with cams, depth, conf and optional rgb."""
        cf, keep = self._frames(frames)
        if outs is None:
            outs = []
            for fr in frames:
                P = sum(int(c.width) * int(c.height) for c in fr["cams"])
                outs.append(Output(P, P, rgb=fr.get("rgb") is not None, members=members))
        co = (ff_output * len(frames))(*[o.c() for o in outs])
        prm = (params or Params()).c
        _check(_lib.ff_fuse_batch(self.h, len(frames), cf, ctypes.byref(prm), co,
                                  _stream_ptr(stream)), "ff_fuse_batch")
        return outs

    def emc(self, cams, depth: Sequence, out: Output, c_occ: float = 0.003, stride: int = 1,
            stream=None) -> Dict:
        """Eq. 12 of the fused cloud in `out` against these depth maps (ff_emc); waits for
        the result: E_MC in metres, points used, mean cameras seeing a used point."""
        torch = _torch()
        ccams, views = self._views(cams, depth, None, None)
        res = torch.zeros(3, dtype=torch.float64, device=out.xyz.device)
        prm = ff_emc_params()
        _lib.ff_emc_params_default(ctypes.byref(prm))
        prm.c_occ, prm.stride = float(c_occ), int(stride)
        _check(_lib.ff_emc(self.h, len(cams), ccams, views, out.xyz.data_ptr(),
                           out.count.data_ptr(), out.capacity, ctypes.byref(prm),
                           res.data_ptr(), _stream_ptr(stream)), "ff_emc")
        r = res.cpu().tolist()
        return dict(emc_m=r[0], points=int(round(r[1])), mean_visible=r[2])

    def tuning_for(self, frames: List[Dict], params: Optional[Params] = None) -> Optional[Dict]:
        """The tuning cached for this batch shape, or None."""
        cf, keep = self._frames(frames)
        t, found = ff_tuning(), ctypes.c_int32()
        _check(_lib.ff_tuning_lookup(self.h, len(frames), cf, ctypes.byref((params or Params()).c),
                                     ctypes.byref(t), ctypes.byref(found)), "ff_tuning_lookup")
        return {k: getattr(t, k) for k, _ in ff_tuning._fields_} if found.value else None

    def export_tuning(self) -> str:
        """The per-shape tuning cache as JSON text (ff_tuning_export)."""
        need = ctypes.c_uint64()
        _lib.ff_tuning_export(self.h, None, 0, ctypes.byref(need))
        buf = ctypes.create_string_buffer(int(need.value))
        _check(_lib.ff_tuning_export(self.h, buf, need.value, ctypes.byref(need)),
               "ff_tuning_export")
        return buf.value.decode()

    def import_tuning(self, text: str) -> int:
        """Merge a JSON tuning cache (entries of other devices are skipped); returns the
        number of entries taken."""
        n = ctypes.c_int32()
        _check(_lib.ff_tuning_import(self.h, text.encode(), ctypes.byref(n)), "ff_tuning_import")
        return int(n.value)

    def save_tuning(self, path: str):
        with open(path, "w") as f:
            f.write(self.export_tuning())

    def load_tuning(self, path: str) -> int:
        with open(path) as f:
            return self.import_tuning(f.read())

    def autotune(self, frames: List[Dict], params: Optional[Params] = None,
                 outs: Optional[List[Output]] = None, stream=None) -> Dict:
        cf, keep = self._frames(frames)
        if outs is None:
            outs = [Output(sum(int(c.width) * int(c.height) for c in fr["cams"]),
                           rgb=fr.get("rgb") is not None) for fr in frames]
        co = (ff_output * len(frames))(*[o.c() for o in outs])
        prm = (params or Params()).c
        t = ff_tuning()
        _check(_lib.ff_autotune(self.h, len(frames), cf, ctypes.byref(prm), co,
                                _stream_ptr(stream), ctypes.byref(t)), "ff_autotune")
        return {k: getattr(t, k) for k, _ in ff_tuning._fields_}


class Server:
    """Continuous-batching server (C++ scheduler thread inside the library).

    submit() queues a frame (device tensors) arriving at `arrival_s` on the server clock;
    results land in the returned Output.  plain=True gives the one-frame-at-a-time baseline."""

    def __init__(self, hbm_budget_bytes: int = 16 << 30, lanes: int = 2,
                 max_batch_frames: int = 16, max_cameras: int = 256, max_pending: int = 4096,
                 plain: bool = False, autotune: bool = False, device: Optional[int] = None):
        torch = _torch()
        if device is None:
            device = torch.cuda.current_device()
        cfg = ff_server_config()
        _lib.ff_server_config_default(ctypes.byref(cfg))
        cfg.hbm_budget_bytes, cfg.lanes = int(hbm_budget_bytes), int(lanes)
        cfg.max_batch_frames, cfg.max_cameras = int(max_batch_frames), int(max_cameras)
        cfg.max_pending, cfg.plain = int(max_pending), int(bool(plain))
        cfg.autotune = int(bool(autotune))
        h = ctypes.c_void_p()
        _check(_lib.ff_server_create(ctypes.byref(h), device, ctypes.byref(cfg)), "ff_server_create")
        self.h = h
        self._keep = {}

    def close(self):
        if getattr(self, "h", None):
            _lib.ff_server_destroy(self.h)
            self.h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def max_pixels(self) -> int:
        """Largest single frame (pixels) the budget admits."""
        return int(_lib.ff_server_max_pixels(self.h))

    def now(self) -> float:
        return float(_lib.ff_server_now(self.h))

    def submit(self, rig: int, frame: Dict, out: "Output", params: Optional[Params] = None,
               arrival_s: Optional[float] = None, stream=None) -> int:
        """Queue a frame; it arrives at `arrival_s` on the server clock (None: now).  Work
        queued on `stream` (default: torch's current stream) before this call is complete
        before the frame is read."""
        ccams, views = Context._views(frame["cams"], frame["depth"], frame.get("conf"),
                                      frame.get("rgb"))
        fr = ff_frame(len(frame["cams"]), ctypes.cast(ccams, ctypes.POINTER(ff_camera)),
                      ctypes.cast(views, ctypes.POINTER(ff_view)))
        o = out.c()
        prm = (params or Params()).c
        t = ctypes.c_uint64()
        a = -1.0 if arrival_s is None else float(arrival_s)
        _check(_lib.ff_server_submit(self.h, int(rig), ctypes.byref(fr), ctypes.byref(prm),
                                     ctypes.byref(o), a, _stream_ptr(stream), ctypes.byref(t)),
               "ff_server_submit")
        self._keep[t.value] = (frame, out)       # device buffers stay alive until done
        return t.value

    def poll(self, ticket: int) -> bool:
        """True once the frame is done (then its status is checked and the ticket is
        forgotten)."""
        d = ctypes.c_int32()
        st = _lib.ff_server_poll(self.h, ticket, ctypes.byref(d))
        if d.value:
            self._keep.pop(ticket, None)
        _check(st, "ff_server_poll")
        return bool(d.value)

    def wait(self, ticket: int):
        st = _lib.ff_server_wait(self.h, ticket)
        self._keep.pop(ticket, None)
        _check(st, "ff_server_wait")

    def drain(self):
        st = _lib.ff_server_drain(self.h)
        self._keep.clear()
        _check(st, "ff_server_drain")

    def stats(self) -> Dict:
        s = ff_stats()
        _check(_lib.ff_server_stats(self.h, ctypes.byref(s)), "ff_server_stats")
        return {k: getattr(s, k) for k, _ in ff_stats._fields_}

    def reset_stats(self):
        _check(_lib.ff_server_reset_stats(self.h), "ff_server_reset_stats")

    def reserve(self, pixels: int, cameras: int, frames: int = 1):
        """Size every idle lane's workspace now for such a batch (ff_server_reserve)."""
        _check(_lib.ff_server_reserve(self.h, int(pixels), int(cameras), int(frames)),
               "ff_server_reserve")

    def latencies(self):
        """(rig ids, latencies in ms) of the frames completed since the last reset, in
        completion order (NumPy arrays)."""
        import numpy as np
        n = ctypes.c_uint64(0)
        _check(_lib.ff_server_latencies(self.h, 0, None, None, ctypes.byref(n)),
               "ff_server_latencies")
        while True:
            cap = n.value
            rigs = np.zeros(cap, np.int32)
            lat = np.zeros(cap, np.float64)
            _check(_lib.ff_server_latencies(
                self.h, cap, rigs.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                lat.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(n)),
                "ff_server_latencies")
            if n.value <= cap:
                return rigs[:n.value], lat[:n.value]

    def probe(self, slot: int):
        """Time trace slot `slot` in every later batch on every lane (-1: off)."""
        _check(_lib.ff_server_probe_enable(self.h, int(slot)), "ff_server_probe_enable")

    def probe_read(self) -> Dict:
        p = ff_probe()
        _check(_lib.ff_server_probe_read(self.h, ctypes.byref(p)), "ff_server_probe_read")
        return _probe_dict(p)


def confidence(cams, depth: Sequence, out: Optional[Sequence] = None, alpha: float = 0.5,
               beta: float = 0.5, gamma: float = 1.0, delta: float = 1.0,
               stream=None) -> List:
    """Eq. 3 confidence maps of the depth maps (ff_confidence), as device tensors."""
    torch = _torch()
    n = len(cams)
    ccams, views = Context._views(cams, depth, None, None)
    if out is None:
        out = [torch.empty_like(d) for d in depth]
    for k, cam in enumerate(cams):
        _check_image(out[k], int(cam.height), int(cam.width), torch.float32, f"out[{k}]")
    ptrs = (ctypes.c_void_p * n)(*[o.data_ptr() for o in out])
    prm = ff_conf_params(alpha, beta, gamma, delta)
    _check(_lib.ff_confidence(n, ccams, views, ptrs, ctypes.byref(prm), _stream_ptr(stream)),
           "ff_confidence")
    return list(out)


def emc_noalloc(cams, depth: Sequence, xyz, count, capacity: int, res, c_occ: float = 0.003,
                stride: int = 1, stream=None):
    """Eq. 12 through ff_emc_noalloc (no context, nothing allocated by the library): the
    fused points `xyz` (device float32 [capacity][3]) with `count` (device uint32/int32 [1])
    against these depth maps; the result goes to `res` (device float64 [3]: E_MC in metres,
    points used, mean cameras seeing a used point).  Asynchronous on `stream`."""
    ccams, views = Context._views(cams, depth, None, None)
    prm = ff_emc_params()
    _lib.ff_emc_params_default(ctypes.byref(prm))
    prm.c_occ, prm.stride = float(c_occ), int(stride)
    _check(_lib.ff_emc_noalloc(len(cams), ccams, views, xyz.data_ptr(), count.data_ptr(),
                               int(capacity), ctypes.byref(prm), res.data_ptr(),
                               _stream_ptr(stream)), "ff_emc_noalloc")
    return res


def to_device(frame, device="cuda", with_rgb=True) -> Dict:
    """Upload a synthetic/host frame (cams, depth, conf, rgb as NumPy) to device tensors."""
    torch = _torch()
    up = lambda a: torch.from_numpy(a).to(device).contiguous()
    d = dict(cams=list(frame.cams), depth=[up(x) for x in frame.depth],
             conf=[up(x) for x in frame.conf])
    if with_rgb and frame.rgb is not None:
        d["rgb"] = [up(x) for x in frame.rgb]
    return d


__all__ = ["Context", "Output", "Params", "Server", "FuseFlowError", "to_device", "version", "lib",
           "FF_NO_MF", "FF_NO_DC", "FF_NO_SA", "FF_CONF_EQ3", "PAD", "EXPORTS", "confidence"]
