"""ctypes binding of libgsr (include/gsr.h): same names, argument marshalling only.

Every step of the render and backward runs in the HIP library; this module
only builds the C structs from torch tensors (device memory) and the torch
stream, and raises GsrError on a non-zero status. It fails loudly when the
library is not built: there is no fallback path.
"""
from __future__ import annotations

import ctypes

import numpy as np
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libgsr.so")

GSR_OK, GSR_EINVAL, GSR_ENOMEM, GSR_EHIP, GSR_ESTATE = 0, -1, -2, -3, -4
GSR_BWD_PLAIN_ATOMIC, GSR_BWD_WAVE_REDUCE, GSR_BWD_SERIAL_REDUCE, GSR_BWD_BLOCK_REDUCE = 0, 1, 2, 3
GSR_BWD_PLAIN_COMPILER_REDUCE = 4
GSR_FLAG_DEBUG_COUNTERS = 1
GSR_FLAG_XCD_REMAP = 2
GSR_FLAG_STAGE_TIMING = 4
GSR_FLAG_LANE_SPLIT_ATOMICS = 8
GSR_FLAG_NO_TILE_ORDER = 16
GSR_FLAG_ACC_F32 = 32
GSR_MAX_BATCH = 16
GSR_EBUDGET = -5
GSR_ACC_STRIDE = 16
GSR_NOALLOC_MAX_GAUSSIANS = 524288
GSR_NOALLOC_MAX_TILES = 65536
(GSR_MB_COPY, GSR_MB_ATOMIC_F32_DISTINCT, GSR_MB_ATOMIC_F64_DISTINCT, GSR_MB_ATOMIC_F32_SAME_ADDRESS,
 GSR_MB_ATOMIC_F32_ONE_LANE, GSR_MB_ATOMIC_F64_NINE_LANES, GSR_MB_WRITE, GSR_MB_READ, GSR_MB_COPY_NT,
 GSR_MB_GATHER48) = range(10)

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
                ("hist", c_uint64 * 65), ("visited", c_uint64), ("max_wave_visits", c_uint64),
                ("walked", c_uint64)]


class gsr_stage_times_t(ctypes.Structure):
    _fields_ = [(name, c_float) for name in ("preprocess", "depth_sort", "scan_emit", "tile_sort", "ranges",
                                             "composite_fwd", "zero_acc", "composite_bwd", "preprocess_bwd")]


class gsr_tune_space(ctypes.Structure):
    _fields_ = [("n_tiles", c_int32), ("tiles", c_int32 * 3), ("n_batches", c_int32), ("batches", c_int32 * 3),
                ("n_thresholds", c_int32), ("thresholds", c_int32 * 12), ("reps", c_int32), ("flags", c_int32)]


class gsr_tune_entry(ctypes.Structure):
    _fields_ = [("config", gsr_config), ("render_ms", ctypes.c_float), ("backward_ms", ctypes.c_float)]


class gsr_server_opts(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", c_int64), ("max_batch", c_int32), ("lanes", c_int32), ("config", gsr_config),
                ("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("capacity_render", c_int32)]


class gsr_request(ctypes.Structure):
    _fields_ = [("scene", c_int32), ("camera", gsr_camera), ("target_seed", ctypes.c_uint64)]


class gsr_result(ctypes.Structure):
    _fields_ = [("id", c_int64), ("scene", c_int32), ("status", c_int32), ("batch_size", c_int32), ("lane", c_int32),
                ("step", c_int32), ("loss", ctypes.c_float), ("t_arrival", ctypes.c_double),
                ("t_start", ctypes.c_double), ("t_done", ctypes.c_double), ("render_mode", c_int32)]


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
    "gsr_backward_noalloc": (c_int32, [c_void_p, c_void_p, c_void_p, ctypes.POINTER(gsr_grads), c_int32,
                                       ctypes.POINTER(gsr_config)]),
    "gsr_render_batch": (c_int32, [c_void_p, c_int32, ctypes.POINTER(gsr_scene), ctypes.POINTER(gsr_camera),
                                   ctypes.POINTER(gsr_config), ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p)]),
    "gsr_backward_batch": (c_int32, [c_void_p, c_int32, ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p),
                                     ctypes.POINTER(gsr_grads), c_int32, ctypes.POINTER(gsr_config)]),
    "gsr_graph_capture_backward": (c_int32, [c_void_p, c_int32, ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p),
                                             ctypes.POINTER(gsr_grads), c_int32, ctypes.POINTER(gsr_config),
                                             ctypes.POINTER(c_void_p)]),
    "gsr_graph_launch": (c_int32, [c_void_p, c_void_p]),
    "gsr_graph_destroy": (None, [c_void_p, c_void_p]),
    "gsr_autotune": (c_int32, [c_void_p, c_int32, ctypes.POINTER(gsr_scene), ctypes.POINTER(gsr_camera),
                               ctypes.POINTER(c_void_p), ctypes.POINTER(gsr_tune_space), ctypes.POINTER(gsr_config),
                               ctypes.POINTER(gsr_tune_entry), c_int32, ctypes.POINTER(c_int32)]),
    "gsr_tuner_create": (c_int32, [ctypes.POINTER(gsr_tune_space), c_int32, ctypes.POINTER(c_void_p)]),
    "gsr_tuner_next": (c_int32, [c_void_p, c_void_p, c_int32, ctypes.POINTER(gsr_scene), ctypes.POINTER(gsr_camera),
                                 ctypes.POINTER(c_void_p), ctypes.POINTER(gsr_config), ctypes.POINTER(c_int32)]),
    "gsr_tuner_destroy": (None, [c_void_p]),
    "gsr_server_scene_bytes": (c_int64, [c_int64, c_int32]),
    "gsr_server_create": (c_int32, [c_int32, ctypes.POINTER(gsr_server_opts), ctypes.POINTER(c_void_p)]),
    "gsr_server_destroy": (None, [c_void_p]),
    "gsr_server_last_error": (ctypes.c_char_p, [c_void_p]),
    "gsr_server_now": (ctypes.c_double, [c_void_p]),
    "gsr_server_add_scene": (c_int32, [c_void_p, ctypes.POINTER(gsr_scene), ctypes.POINTER(c_int32)]),
    "gsr_server_remove_scene": (c_int32, [c_void_p, c_int32]),
    "gsr_server_scene_state": (c_int32, [c_void_p, c_int32, ctypes.POINTER(gsr_scene), ctypes.POINTER(gsr_grads),
                                         ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p), ctypes.POINTER(c_int32)]),
    "gsr_server_set_step": (c_int32, [c_void_p, c_int32, c_int32]),
    "gsr_server_scene_io": (c_int32, [c_void_p, c_int32, c_int32, c_void_p, c_int32]),
    "gsr_server_submit": (c_int32, [c_void_p, ctypes.POINTER(gsr_request), ctypes.POINTER(c_int64)]),
    "gsr_server_replay": (c_int32, [c_void_p, c_int32, ctypes.POINTER(gsr_request), ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(c_int64)]),
    "gsr_server_drain": (c_int32, [c_void_p]),
    "gsr_server_results": (c_int32, [c_void_p, ctypes.POINTER(gsr_result), c_int32, ctypes.POINTER(c_int32)]),
    "gsr_l1_dssim_grad": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_int32, ctypes.c_float, c_void_p,
                                    c_void_p]),
    "gsr_rerender_batch": (c_int32, [c_void_p, c_int32, ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p),
                                     ctypes.POINTER(gsr_config)]),
    "gsr_fwd_sync": (c_int32, [c_void_p, c_void_p, ctypes.POINTER(c_int64), ctypes.POINTER(c_int32)]),
    "gsr_graph_capture_step": (c_int32, [c_void_p, c_int32, ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p),
                                         ctypes.POINTER(c_void_p), ctypes.c_float, ctypes.POINTER(c_void_p),
                                         ctypes.POINTER(gsr_grads), c_int32, ctypes.POINTER(gsr_config),
                                         ctypes.POINTER(c_void_p)]),
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
    "gsr_microbench": (c_int32, [c_void_p, c_int32, c_int64, c_int32, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_double)]),
}


def load(path: str = LIB_PATH):
    """Load libgsr.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libgsr is not built ({path} missing); run python -m paper_2401_05345_amd.build")
    try:
        # torch first: its wheel brings its own HIP runtime, and the library must bind to that one
        # (loaded the other way round, both runtimes end up in the process and context creation
        # fails).
        import torch  # noqa: F401
    except ImportError:
        pass
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


def gsr_backward_noalloc(ctx, state, dl_dimage, grads: gsr_grads, accumulate: int = 0,
                         cfg: gsr_config | None = None):
    _check(ctx, load().gsr_backward_noalloc(ctx, state, _ptr(dl_dimage), ctypes.byref(grads), int(accumulate),
                                            ctypes.byref(cfg) if cfg is not None else None))


def gsr_render_batch(ctx, scenes, cams, cfg: gsr_config, images):
    """Render len(scenes) views in one call; returns the list of their states."""
    n = len(scenes)
    states = (c_void_p * n)()
    _check(ctx, load().gsr_render_batch(ctx, n, (gsr_scene * n)(*scenes), (gsr_camera * n)(*cams),
                                        ctypes.byref(cfg), (c_void_p * n)(*[im.data_ptr() for im in images]),
                                        states))
    return [c_void_p(s) for s in states]


def gsr_backward_batch(ctx, states, dl_dimages, grads, accumulate: int = 0, cfg: gsr_config | None = None):
    n = len(states)
    _check(ctx, load().gsr_backward_batch(ctx, n, (c_void_p * n)(*[s.value for s in states]),
                                          (c_void_p * n)(*[d.data_ptr() for d in dl_dimages]),
                                          (gsr_grads * n)(*grads), int(accumulate),
                                          ctypes.byref(cfg) if cfg is not None else None))


def gsr_graph_capture_backward(ctx, states, dl_dimages, grads, accumulate: int = 0, cfg: gsr_config | None = None):
    n = len(states)
    graph = c_void_p()
    _check(ctx, load().gsr_graph_capture_backward(ctx, n, (c_void_p * n)(*[s.value for s in states]),
                                                  (c_void_p * n)(*[d.data_ptr() for d in dl_dimages]),
                                                  (gsr_grads * n)(*grads), int(accumulate),
                                                  ctypes.byref(cfg) if cfg is not None else None,
                                                  ctypes.byref(graph)))
    return graph


def gsr_rerender_batch(ctx, states, images, cfg: gsr_config | None = None):
    n = len(states)
    _check(ctx, load().gsr_rerender_batch(ctx, n, (c_void_p * n)(*[s.value for s in states]),
                                          (c_void_p * n)(*[im.data_ptr() for im in images]),
                                          ctypes.byref(cfg) if cfg is not None else None))


def gsr_fwd_sync(ctx, state):
    """Returns (pair count, overflowed)."""
    p, o = c_int64(), c_int32()
    _check(ctx, load().gsr_fwd_sync(ctx, state, ctypes.byref(p), ctypes.byref(o)))
    return p.value, bool(o.value)


def gsr_graph_capture_step(ctx, states, images, targets, dl_dimages, grads, lam: float = 0.0, accumulate: int = 0,
                           cfg: gsr_config | None = None):
    n = len(states)
    graph = c_void_p()
    ptrs = lambda ts: (c_void_p * n)(*[t.data_ptr() for t in ts])
    _check(ctx, load().gsr_graph_capture_step(ctx, n, (c_void_p * n)(*[s.value for s in states]), ptrs(images),
                                              ptrs(targets), float(lam), ptrs(dl_dimages), (gsr_grads * n)(*grads),
                                              int(accumulate), ctypes.byref(cfg) if cfg is not None else None,
                                              ctypes.byref(graph)))
    return graph


def gsr_graph_launch(ctx, graph):
    _check(ctx, load().gsr_graph_launch(ctx, graph))


def gsr_graph_destroy(ctx, graph):
    load().gsr_graph_destroy(ctx, graph)


def make_tune_space(tiles=(8, 16, 32), batches=(64, 128, 256), thresholds=(1, 2, 4, 8, 16, 24, 32, 48, 64), reps=3,
                    flags=0) -> gsr_tune_space:
    """Candidate space of the autotuner. The default thresholds are the paper's 8..64 range plus
    1, 2 and 4, where the optimum lies on MI355X (each plain lane-atomic is a fabric request)."""
    sp = gsr_tune_space()
    sp.n_tiles, sp.n_batches, sp.n_thresholds = len(tiles), len(batches), len(thresholds)
    for i, v in enumerate(tiles):
        sp.tiles[i] = v
    for i, v in enumerate(batches):
        sp.batches[i] = v
    for i, v in enumerate(thresholds):
        sp.thresholds[i] = v
    sp.reps, sp.flags = reps, flags
    return sp


def _dl_array(n, dl_dimages):
    if dl_dimages is None:
        return None
    return (c_void_p * n)(*[None if d is None else d.data_ptr() for d in dl_dimages])


def gsr_autotune(ctx, scenes, cams, space: gsr_tune_space, dl_dimages=None, max_entries=64):
    """Returns (best config, list of gsr_tune_entry)."""
    n = len(scenes)
    best = gsr_config()
    entries = (gsr_tune_entry * max_entries)()
    count = c_int32()
    _check(ctx, load().gsr_autotune(ctx, n, (gsr_scene * n)(*scenes), (gsr_camera * n)(*cams),
                                    _dl_array(n, dl_dimages), ctypes.byref(space), ctypes.byref(best), entries,
                                    max_entries, ctypes.byref(count)))
    return best, list(entries[: count.value])


def gsr_tuner_create(space: gsr_tune_space, every: int):
    t = c_void_p()
    st = load().gsr_tuner_create(ctypes.byref(space), int(every), ctypes.byref(t))
    if st != GSR_OK:
        raise GsrError(st, "gsr_tuner_create: invalid space or period")
    return t


def gsr_tuner_next(ctx, tuner, scenes, cams, dl_dimages=None):
    """Returns (config for this iteration, whether it re-tuned)."""
    n = len(scenes)
    cfg = gsr_config()
    did = c_int32()
    _check(ctx, load().gsr_tuner_next(ctx, tuner, n, (gsr_scene * n)(*scenes), (gsr_camera * n)(*cams),
                                      _dl_array(n, dl_dimages), ctypes.byref(cfg), ctypes.byref(did)))
    return cfg, bool(did.value)


def gsr_tuner_destroy(tuner):
    load().gsr_tuner_destroy(tuner)


# ---------------------------------------------------------------- serving

def _scheck(server, status):
    if status != GSR_OK:
        msg = _lib.gsr_server_last_error(server).decode() if server else ""
        raise GsrError(status, msg)


def make_server_opts(budget_bytes, max_batch=16, lanes=2, config=None, lr=1e-3, beta1=0.9, beta2=0.999,
                     eps=1e-15, capacity_render=0) -> gsr_server_opts:
    return gsr_server_opts(int(budget_bytes), max_batch, lanes, config if config is not None else make_config(),
                           lr, beta1, beta2, eps, int(capacity_render))


def gsr_server_scene_bytes(n: int, sh_degree: int) -> int:
    return int(load().gsr_server_scene_bytes(n, sh_degree))


def gsr_server_create(opts: gsr_server_opts, device: int = 0):
    srv = c_void_p()
    st = load().gsr_server_create(device, ctypes.byref(opts), ctypes.byref(srv))
    if st != GSR_OK:
        raise GsrError(st, "gsr_server_create failed")
    return srv


def gsr_server_destroy(server):
    load().gsr_server_destroy(server)


def gsr_server_now(server) -> float:
    return float(load().gsr_server_now(server))


def gsr_server_add_scene(server, scene: gsr_scene) -> int:
    sid = c_int32()
    _scheck(server, load().gsr_server_add_scene(server, ctypes.byref(scene), ctypes.byref(sid)))
    return sid.value


def gsr_server_remove_scene(server, sid: int):
    _scheck(server, load().gsr_server_remove_scene(server, sid))


def gsr_server_scene_state(server, sid: int):
    """Returns (params gsr_scene, grads gsr_grads, adam_m ptr, adam_v ptr, step)."""
    p, g, m, v, step = gsr_scene(), gsr_grads(), c_void_p(), c_void_p(), c_int32()
    _scheck(server, load().gsr_server_scene_state(server, sid, ctypes.byref(p), ctypes.byref(g), ctypes.byref(m),
                                                  ctypes.byref(v), ctypes.byref(step)))
    return p, g, m.value, v.value, step.value


def gsr_server_set_step(server, sid: int, step: int):
    _scheck(server, load().gsr_server_set_step(server, sid, step))


SCENE_BLOCKS = ("params", "grads", "adam_m", "adam_v")


def gsr_server_scene_io(server, sid: int, block: str, host: np.ndarray, to_host: bool):
    """Copy a scene's flat block to/from the contiguous fp32 numpy array `host`."""
    assert host.dtype == np.float32 and host.flags.c_contiguous
    _scheck(server, load().gsr_server_scene_io(server, sid, SCENE_BLOCKS.index(block),
                                               host.ctypes.data_as(c_void_p), 1 if to_host else 0))


def gsr_server_submit(server, req: gsr_request) -> int:
    rid = c_int64()
    _scheck(server, load().gsr_server_submit(server, ctypes.byref(req), ctypes.byref(rid)))
    return rid.value


def gsr_server_replay(server, reqs, arrival_s):
    n = len(reqs)
    ids = (c_int64 * n)()
    _scheck(server, load().gsr_server_replay(server, n, (gsr_request * n)(*reqs),
                                             (ctypes.c_double * n)(*[float(t) for t in arrival_s]), ids))
    return list(ids)


def gsr_server_drain(server):
    _scheck(server, load().gsr_server_drain(server))


def gsr_server_results(server, max_results: int = 4096):
    out = (gsr_result * max_results)()
    n = c_int32()
    _scheck(server, load().gsr_server_results(server, out, max_results, ctypes.byref(n)))
    return list(out[: n.value])


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


def gsr_l1_dssim_grad(ctx, image, target, dl_dimage, lam: float = 0.2, loss=None):
    _, h, w = image.shape
    _check(ctx, load().gsr_l1_dssim_grad(ctx, _ptr(image), _ptr(target), h, w, float(lam), _ptr(dl_dimage),
                                         _ptr(loss)))


def gsr_wave_reduce_selftest(ctx, vals, active, mode, threshold, lane_split, sums, lane_atomics):
    n_waves = int(active.numel() // 64)
    _check(ctx, load().gsr_wave_reduce_selftest(ctx, _ptr(vals), _ptr(active), n_waves, int(mode), int(threshold),
                                                int(lane_split), _ptr(sums), _ptr(lane_atomics)))


def gsr_microbench(ctx, kind: int, nbytes: int, reps: int = 5):
    """(median ms per launch, operations per launch) of one GSR_MB_* pattern."""
    ms, ops = ctypes.c_double(), ctypes.c_double()
    _check(ctx, load().gsr_microbench(ctx, int(kind), int(nbytes), int(reps), ctypes.byref(ms), ctypes.byref(ops)))
    return ms.value, ops.value


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
