"""ctypes binding of libgsr (include/gsr.h): same names, argument marshalling only.

Every step of the render and backward runs in the HIP library; this module
only builds the C structs from torch tensors (device memory) and the torch
stream, and raises GsrError on a non-zero status. It fails loudly when the
library is not built: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libgsr.so")

GSR_OK, GSR_EINVAL, GSR_ENOMEM, GSR_EHIP, GSR_ESTATE = 0, -1, -2, -3, -4
GSR_BWD_PLAIN_ATOMIC, GSR_BWD_WAVE_REDUCE = 0, 1
GSR_FLAG_DEBUG_COUNTERS = 1
GSR_FLAG_XCD_REMAP = 2
GSR_FLAG_STAGE_TIMING = 4
GSR_FLAG_LANE_SPLIT_ATOMICS = 8
GSR_FLAG_NO_TILE_ORDER = 16
GSR_ACC_STRIDE = 16

c_void_p = ctypes.c_void_p
c_int32 = ctypes.c_int32
c_int64 = ctypes.c_int64
c_float = ctypes.c_float
c_uint64 = ctypes.c_uint64


class gsr_scene(ctypes.Structure):
    _fields_ = [("n", c_int32), ("sh_degree", c_int32), ("means3d", c_void_p), ("log_scales", c_void_p),
                ("quats", c_void_p), ("opacity_logits", c_void_p), ("sh", c_void_p)]


class gsr_camera(ctypes.Structure):
    _fields_ = [("width", c_int32), ("height", c_int32), ("fx", c_float), ("fy", c_float), ("cx", c_float),
                ("cy", c_float), ("world_to_cam", c_float * 12), ("znear", c_float), ("bg", c_float * 3)]


class gsr_config(ctypes.Structure):
    _fields_ = [("tile", c_int32), ("lds_batch", c_int32), ("bwd_mode", c_int32), ("reduce_threshold", c_int32),
                ("flags", c_int32)]


class gsr_grads(ctypes.Structure):
    _fields_ = [("means3d", c_void_p), ("log_scales", c_void_p), ("quats", c_void_p),
                ("opacity_logits", c_void_p), ("sh", c_void_p)]


class gsr_fwd_stats_t(ctypes.Structure):
    _fields_ = [("n", c_int64), ("n_visible", c_int64), ("n_pairs", c_int64), ("grid_x", c_int32),
                ("grid_y", c_int32), ("tile", c_int32)]


class gsr_fwd_export_t(ctypes.Structure):
    _fields_ = [(name, c_void_p) for name in ("mean2d", "conic_opacity", "rgb", "depth", "radius", "tiles_touched",
                                              "clamp_mask", "sorted_ids", "ranges", "T_final", "n_contrib", "acc")]


class gsr_bwd_counters_t(ctypes.Structure):
    _fields_ = [("evaluated", c_uint64), ("active", c_uint64), ("wave_entries", c_uint64), ("reduced", c_uint64),
                ("plain_lanes", c_uint64), ("lane_atomics", c_uint64), ("atomic_instrs", c_uint64),
                ("hist", c_uint64 * 65)]


class gsr_stage_times_t(ctypes.Structure):
    _fields_ = [(name, c_float) for name in ("preprocess", "depth_sort", "scan_emit", "tile_sort", "ranges",
                                             "composite_fwd", "zero_acc", "composite_bwd", "preprocess_bwd")]


class GsrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"gsr status {status}: {msg}")
        self.status = status


_lib = None

_PROTOS = {
    "gsr_version": (ctypes.c_char_p, []),
    "gsr_validate_scene": (c_int32, [ctypes.POINTER(gsr_scene)]),
    "gsr_validate_camera": (c_int32, [ctypes.POINTER(gsr_camera)]),
    "gsr_validate_config": (c_int32, [ctypes.POINTER(gsr_config), ctypes.POINTER(gsr_camera)]),
    "gsr_ctx_create": (c_int32, [ctypes.POINTER(c_void_p), c_int32, c_void_p]),
    "gsr_ctx_destroy": (None, [c_void_p]),
    "gsr_ctx_last_error": (ctypes.c_char_p, [c_void_p]),
    "gsr_ctx_set_stream": (c_int32, [c_void_p, c_void_p]),
    "gsr_render": (c_int32, [c_void_p, ctypes.POINTER(gsr_scene), ctypes.POINTER(gsr_camera),
                             ctypes.POINTER(gsr_config), c_void_p, ctypes.POINTER(c_void_p)]),
    "gsr_backward": (c_int32, [c_void_p, c_void_p, c_void_p, ctypes.POINTER(gsr_grads), c_int32,
                               ctypes.POINTER(gsr_config)]),
    "gsr_backward_composite": (c_int32, [c_void_p, c_void_p, c_void_p, ctypes.POINTER(gsr_config)]),
    "gsr_backward_params": (c_int32, [c_void_p, c_void_p, ctypes.POINTER(gsr_grads), c_int32]),
    "gsr_fwd_release": (c_int32, [c_void_p, c_void_p]),
    "gsr_fwd_stats": (c_int32, [c_void_p, ctypes.POINTER(gsr_fwd_stats_t)]),
    "gsr_fwd_export": (c_int32, [c_void_p, c_void_p, ctypes.POINTER(gsr_fwd_export_t)]),
    "gsr_bwd_counters": (c_int32, [c_void_p, c_void_p, ctypes.POINTER(gsr_bwd_counters_t)]),
    "gsr_ctx_stage_times": (c_int32, [c_void_p, ctypes.POINTER(gsr_stage_times_t)]),
    "gsr_l1_grad": (c_int32, [c_void_p, c_void_p, c_void_p, c_int64, c_void_p]),
    "gsr_wave_reduce_selftest": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_int32, c_int32, c_int32,
                                           c_void_p, c_void_p]),
}


def load(path: str = LIB_PATH):
    """Load libgsr.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libgsr is not built ({path} missing); run python -m paper_2401_05345_amd.build")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _PROTOS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(ctx, status):
    if status != GSR_OK:
        msg = _lib.gsr_ctx_last_error(ctx).decode() if ctx else ""
        raise GsrError(status, msg)


# ---------------------------------------------------------------- helpers

def _ptr(t):
    return None if t is None else c_void_p(t.data_ptr())


def make_scene(means3d, log_scales, quats, opacity_logits, sh, sh_degree: int) -> gsr_scene:
    for t in (means3d, log_scales, quats, opacity_logits, sh):
        if t.dtype.itemsize != 4 or not t.is_contiguous():
            raise ValueError("scene tensors must be contiguous fp32")
    return gsr_scene(int(means3d.shape[0]), int(sh_degree), _ptr(means3d), _ptr(log_scales), _ptr(quats),
                     _ptr(opacity_logits), _ptr(sh))


def make_camera(width, height, fx, fy, cx, cy, world_to_cam, znear=0.2, bg=(0.0, 0.0, 0.0)) -> gsr_camera:
    w = [float(x) for x in list(__import__("numpy").asarray(world_to_cam, dtype="float32").reshape(-1))]
    return gsr_camera(int(width), int(height), float(fx), float(fy), float(cx), float(cy), (c_float * 12)(*w),
                      float(znear), (c_float * 3)(*[float(b) for b in bg]))


def make_config(tile=16, lds_batch=256, bwd_mode=GSR_BWD_WAVE_REDUCE, reduce_threshold=32, flags=0) -> gsr_config:
    return gsr_config(int(tile), int(lds_batch), int(bwd_mode), int(reduce_threshold), int(flags))


def make_grads(means3d, log_scales, quats, opacity_logits, sh) -> gsr_grads:
    return gsr_grads(_ptr(means3d), _ptr(log_scales), _ptr(quats), _ptr(opacity_logits), _ptr(sh))


# ---------------------------------------------------------------- same-name wrappers

def gsr_version() -> str:
    return load().gsr_version().decode()


def gsr_validate_scene(scene: gsr_scene) -> int:
    return load().gsr_validate_scene(ctypes.byref(scene))


def gsr_validate_camera(cam: gsr_camera) -> int:
    return load().gsr_validate_camera(ctypes.byref(cam))


def gsr_validate_config(cfg: gsr_config, cam: gsr_camera | None = None) -> int:
    return load().gsr_validate_config(ctypes.byref(cfg), ctypes.byref(cam) if cam is not None else None)


def gsr_ctx_create(device: int = 0, stream=None):
    lib = load()
    out = c_void_p()
    st = lib.gsr_ctx_create(ctypes.byref(out), int(device), c_void_p(stream) if stream else None)
    if st != GSR_OK:
        raise GsrError(st, "gsr_ctx_create failed")
    return out


def gsr_ctx_destroy(ctx):
    load().gsr_ctx_destroy(ctx)


def gsr_ctx_last_error(ctx) -> str:
    return load().gsr_ctx_last_error(ctx).decode()


def gsr_ctx_set_stream(ctx, stream):
    _check(ctx, load().gsr_ctx_set_stream(ctx, c_void_p(stream) if stream else None))


def gsr_render(ctx, scene: gsr_scene, cam: gsr_camera, cfg: gsr_config, image):
    state = c_void_p()
    _check(ctx, load().gsr_render(ctx, ctypes.byref(scene), ctypes.byref(cam), ctypes.byref(cfg), _ptr(image),
                                  ctypes.byref(state)))
    return state


def gsr_backward(ctx, state, dl_dimage, grads: gsr_grads, accumulate: int = 0, cfg: gsr_config | None = None):
    _check(ctx, load().gsr_backward(ctx, state, _ptr(dl_dimage), ctypes.byref(grads), int(accumulate),
                                    ctypes.byref(cfg) if cfg is not None else None))


def gsr_backward_composite(ctx, state, dl_dimage, cfg: gsr_config | None = None):
    _check(ctx, load().gsr_backward_composite(ctx, state, _ptr(dl_dimage),
                                              ctypes.byref(cfg) if cfg is not None else None))


def gsr_backward_params(ctx, state, grads: gsr_grads, accumulate: int = 0):
    _check(ctx, load().gsr_backward_params(ctx, state, ctypes.byref(grads), int(accumulate)))


def gsr_fwd_release(ctx, state):
    _check(ctx, load().gsr_fwd_release(ctx, state))


def gsr_fwd_stats(state) -> gsr_fwd_stats_t:
    out = gsr_fwd_stats_t()
    st = load().gsr_fwd_stats(state, ctypes.byref(out))
    if st != GSR_OK:
        raise GsrError(st, "gsr_fwd_stats failed")
    return out


def gsr_fwd_export(ctx, state, **dst):
    ex = gsr_fwd_export_t()
    for k, v in dst.items():
        setattr(ex, k, None if v is None else v.data_ptr())
    _check(ctx, load().gsr_fwd_export(ctx, state, ctypes.byref(ex)))


def gsr_bwd_counters(ctx, state) -> gsr_bwd_counters_t:
    out = gsr_bwd_counters_t()
    _check(ctx, load().gsr_bwd_counters(ctx, state, ctypes.byref(out)))
    return out


def gsr_ctx_stage_times(ctx) -> gsr_stage_times_t:
    out = gsr_stage_times_t()
    _check(ctx, load().gsr_ctx_stage_times(ctx, ctypes.byref(out)))
    return out


def gsr_l1_grad(ctx, image, target, dl_dimage):
    _check(ctx, load().gsr_l1_grad(ctx, _ptr(image), _ptr(target), int(image.numel()), _ptr(dl_dimage)))


def gsr_wave_reduce_selftest(ctx, vals, active, mode, threshold, lane_split, sums, lane_atomics):
    n_waves = int(active.numel() // 64)
    _check(ctx, load().gsr_wave_reduce_selftest(ctx, _ptr(vals), _ptr(active), n_waves, int(mode), int(threshold),
                                                int(lane_split), _ptr(sums), _ptr(lane_atomics)))


# ---------------------------------------------------------------- convenience for torch callers

@dataclass
class Frame:
    """Result of a render: image plus the library-owned forward state."""
    image: object
    state: object
    stats: gsr_fwd_stats_t


class Renderer:
    """One context on the current torch device and stream (memory and streams only)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        load()
        self.torch = torch
        self.device = device
        self._stream = stream if stream is not None else torch.cuda.current_stream(device).cuda_stream
        self.ctx = gsr_ctx_create(device, self._stream)

    def close(self):
        if self.ctx:
            gsr_ctx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def scene_from(self, tensors: dict, sh_degree: int) -> gsr_scene:
        return make_scene(tensors["means3d"], tensors["log_scales"], tensors["quats"], tensors["opacity_logits"],
                          tensors["sh"], sh_degree)

    def render(self, scene: gsr_scene, cam: gsr_camera, cfg: gsr_config) -> Frame:
        img = self.torch.empty((3, cam.height, cam.width), device=f"cuda:{self.device}", dtype=self.torch.float32)
        st = gsr_render(self.ctx, scene, cam, cfg, img)
        return Frame(img, st, gsr_fwd_stats(st))

    def backward(self, frame: Frame, dl_dimage, grads: gsr_grads, accumulate=0, cfg=None):
        gsr_backward(self.ctx, frame.state, dl_dimage, grads, accumulate, cfg)

    def release(self, frame: Frame):
        if frame.state:
            gsr_fwd_release(self.ctx, frame.state)
            frame.state = None
