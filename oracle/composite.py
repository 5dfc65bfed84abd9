"""fp64 oracle: tile binning and the per-pixel composite (forward and backward).

TEST INFRASTRUCTURE ONLY (tests/, the smoke check and the CPU baseline leg of
the benchmark). Shares no code with the HIP path.

Binning follows the tile-based rasteriser of 3D Gaussian Splatting that the
paper instruments (Background, "Differentiable Rendering for Rasterization
Pipelines"; the gradient kernel consumes a per-pixel list of primitives,
Motivation, "Atomic Reduction Bottleneck"): every visible Gaussian is listed
in each tile of its rectangle, and each tile's list is ordered by ascending
fp32 depth, ties by ascending Gaussian index. The sort is numpy's lexsort
(a library primitive); the per-pixel loops are plain C in raster.c.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

from .preprocess import Projected, project, params_backward

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "raster.c")
_LIB = os.path.join(_HERE, "_build", "liboracle_raster.so")


def build_raster_lib(force: bool = False) -> str:
    """Compile raster.c with gcc (plain -O2, no fast-math, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        os.makedirs(os.path.dirname(_LIB), exist_ok=True)
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
                        "-fno-fast-math", "-fopenmp", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Frame(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int32), ("height", ctypes.c_int32), ("tile", ctypes.c_int32),
        ("grid_x", ctypes.c_int32), ("grid_y", ctypes.c_int32),
        ("tile_start", ctypes.c_void_p), ("ids", ctypes.c_void_p),
        ("mean2d", ctypes.c_void_p), ("conic", ctypes.c_void_p), ("opacity", ctypes.c_void_p),
        ("rgb", ctypes.c_void_p), ("bg", ctypes.c_double * 3), ("tile_select", ctypes.c_void_p),
    ]


_lib = None


def default_threads() -> int:
    """OpenMP threads of the per-pixel loops: OMP_NUM_THREADS when set, else the CPUs this
    process may run on, at most 16."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _raster():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build_raster_lib())
        lib.oracle_render.argtypes = [ctypes.POINTER(_Frame)] + [ctypes.c_void_p] * 6 + [ctypes.c_int]
        lib.oracle_render.restype = ctypes.c_int
        lib.oracle_backward.argtypes = [ctypes.POINTER(_Frame), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                        ctypes.c_int]
        lib.oracle_backward.restype = ctypes.c_int
        lib.oracle_pixel_entries.argtypes = [ctypes.POINTER(_Frame), ctypes.c_int, ctypes.c_int,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
        lib.oracle_pixel_entries.restype = ctypes.c_int64
        _lib = lib
    return _lib


@dataclass
class TileLists:
    tile_start: np.ndarray   # int64 [tiles+1]
    ids: np.ndarray          # int32 [P]
    tile_of: np.ndarray      # int64 [P] tile id per sorted entry
    emitted_gid: np.ndarray  # int64 [P] Gaussian per pair in emission order (by Gaussian, rect row-major)
    emitted_tile: np.ndarray # int64 [P]


def tile_lists(proj: Projected, tile_select: np.ndarray | None = None) -> TileLists:
    """(tile, Gaussian) pairs of every visible Gaussian's rectangle, ordered by (tile, depth, index)."""
    gx, gy = proj.grid
    vis = np.nonzero(proj.visible)[0]
    counts = proj.tiles_touched[vis]
    total = int(counts.sum())
    gid = np.repeat(vis, counts)
    first = np.repeat(np.cumsum(counts) - counts, counts)
    k = np.arange(total, dtype=np.int64) - first
    x_lo, x_hi, y_lo, y_hi = (proj.rect[gid, i] for i in range(4))
    w = x_hi - x_lo
    tx = x_lo + k % np.maximum(w, 1)
    ty = y_lo + k // np.maximum(w, 1)
    tile = ty * gx + tx
    if tile_select is not None:
        keep = tile_select[tile].astype(bool)
        e_gid, e_tile = gid, tile
        gid, tile = gid[keep], tile[keep]
    else:
        e_gid, e_tile = gid, tile
    order = np.lexsort((gid, proj.depth_key[gid], tile))
    ids = gid[order].astype(np.int32)
    ts = tile[order]
    start = np.searchsorted(ts, np.arange(gx * gy + 1), side="left").astype(np.int64)
    return TileLists(start, ids, ts, e_gid, e_tile)


@dataclass
class RenderResult:
    image: np.ndarray      # f64 [3,H,W]
    T_final: np.ndarray    # f64 [H,W]
    n_contrib: np.ndarray  # int32 [H,W]
    margin: np.ndarray     # f64 [H,W] min relative distance of any per-pixel decision to its threshold
    signature: np.ndarray  # uint64 [H,W] hash of the composited entries and their clamp states
    n_used: np.ndarray     # int32 [H,W] number of composited entries
    proj: Projected
    lists: TileLists
    cam: object
    tile: int
    tile_select: np.ndarray | None


def _frame(proj: Projected, lists: TileLists, cam, tile, tile_select, keep):
    gx, gy = proj.grid
    arrs = dict(
        tile_start=np.ascontiguousarray(lists.tile_start, np.int64),
        ids=np.ascontiguousarray(lists.ids, np.int32),
        mean2d=np.ascontiguousarray(proj.mean2d, np.float64),
        conic=np.ascontiguousarray(proj.conic, np.float64),
        opacity=np.ascontiguousarray(proj.opacity, np.float64),
        rgb=np.ascontiguousarray(proj.rgb, np.float64),
    )
    sel = None if tile_select is None else np.ascontiguousarray(tile_select, np.uint8)
    keep.extend(arrs.values())
    keep.append(sel)
    f = _Frame(int(cam.width), int(cam.height), int(tile), int(gx), int(gy),
               arrs["tile_start"].ctypes.data, arrs["ids"].ctypes.data, arrs["mean2d"].ctypes.data,
               arrs["conic"].ctypes.data, arrs["opacity"].ctypes.data, arrs["rgb"].ctypes.data,
               (ctypes.c_double * 3)(*[float(np.float32(b)) for b in cam.bg]),
               None if sel is None else sel.ctypes.data)
    return f


def render(scene, cam, tile: int = 16, tile_select: np.ndarray | None = None,
           threads: int | None = None) -> RenderResult:
    """Forward pass: image [3,H,W] = sum_k alpha_k T_k c_k + T_final bg per pixel."""
    proj = project(scene, cam, tile)
    lists = tile_lists(proj, tile_select)
    H, W = int(cam.height), int(cam.width)
    image = np.zeros((3, H, W))
    T_final = np.ones((H, W))
    n_contrib = np.zeros((H, W), np.int32)
    margin = np.full((H, W), np.inf)
    sig = np.zeros((H, W), np.uint64)
    used = np.zeros((H, W), np.int32)
    keep = []
    f = _frame(proj, lists, cam, tile, tile_select, keep)
    rc = _raster().oracle_render(ctypes.byref(f), image.ctypes.data, T_final.ctypes.data,
                                 n_contrib.ctypes.data, margin.ctypes.data, sig.ctypes.data, used.ctypes.data,
                                 threads or default_threads())
    assert rc == 0
    return RenderResult(image, T_final, n_contrib, margin, sig, used, proj, lists, cam, tile, tile_select)


def composite_backward(rr: RenderResult, dl_dimage: np.ndarray, threads: int | None = None) -> np.ndarray:
    """acc9 [n,9]: per-Gaussian dL/d(mean2d x,y, conic A,B,C, opacity, rgb) summed over pixels."""
    n = rr.proj.n
    acc = np.zeros((n, 9))
    g = np.ascontiguousarray(dl_dimage, np.float64)
    keep = []
    f = _frame(rr.proj, rr.lists, rr.cam, rr.tile, rr.tile_select, keep)
    longest = int(np.max(np.diff(rr.lists.tile_start))) if rr.lists.tile_start.size > 1 else 1
    rc = _raster().oracle_backward(ctypes.byref(f), g.ctypes.data, acc.ctypes.data, max(longest, 1),
                                   threads or default_threads())
    assert rc == 0
    return acc


def backward(scene, rr: RenderResult, dl_dimage: np.ndarray, threads: int | None = None):
    """Full backward: (acc9, [dL/dmeans3d, dL/dlog_scales, dL/dquats, dL/dopacity_logits, dL/dsh])."""
    acc = composite_backward(rr, dl_dimage, threads)
    return acc, params_backward(scene, rr.cam, rr.proj, acc)


def pixel_entries(rr: RenderResult, x: int, y: int):
    """(1-based list positions, Gaussian ids) of the entries composited at pixel (x, y)."""
    keep = []
    f = _frame(rr.proj, rr.lists, rr.cam, rr.tile, rr.tile_select, keep)
    cap = int(np.max(np.diff(rr.lists.tile_start))) + 1
    pos = np.zeros(cap, np.int64)
    ids = np.zeros(cap, np.int32)
    n = _raster().oracle_pixel_entries(ctypes.byref(f), x, y, pos.ctypes.data, ids.ctypes.data, cap)
    return pos[:n], ids[:n]
