"""The C-ABI library loads on a machine without a GPU, exports every function
include/gsr.h declares, and its host-only argument checks behave (no device
calls are made here)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2401_05345_amd import gsr
from paper_2401_05345_amd import scenegen as sg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "gsr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(gsr_[a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(gsr.LIB_PATH):
        from paper_2401_05345_amd import build
        build.build()
    return gsr.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("gsr_ctx_create", "gsr_render", "gsr_backward", "gsr_fwd_release", "gsr_validate_scene",
                 "gsr_wave_reduce_selftest", "gsr_fwd_export", "gsr_bwd_counters", "gsr_render_batch",
                 "gsr_backward_batch"):
        assert must in names
    assert len(names) >= 21


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(declared_functions()) <= set(gsr._PROTOS), "binding lacks a prototype"


def test_version(lib):
    assert "gfx950" in gsr.gsr_version()


def _cam(**kw):
    c = sg.make_camera(64, 48, (0.0, 0.0, -3.0))
    cam = gsr.make_camera(c.width, c.height, c.fx, c.fy, c.cx, c.cy, c.world_to_cam)
    for k, v in kw.items():
        setattr(cam, k, v)
    return cam


def test_validate_camera(lib):
    assert gsr.gsr_validate_camera(_cam()) == gsr.GSR_OK
    assert gsr.gsr_validate_camera(_cam(width=0)) == gsr.GSR_EINVAL
    assert gsr.gsr_validate_camera(_cam(fx=float("nan"))) == gsr.GSR_EINVAL
    assert gsr.gsr_validate_camera(_cam(fy=-1.0)) == gsr.GSR_EINVAL
    assert gsr.gsr_validate_camera(_cam(znear=0.0)) == gsr.GSR_EINVAL
    bad = _cam()
    bad.world_to_cam[0] = 2.0          # not a rotation
    assert gsr.gsr_validate_camera(bad) == gsr.GSR_EINVAL


def test_validate_scene(lib):
    ok = gsr.gsr_scene(0, 0, None, None, None, None, None)
    assert gsr.gsr_validate_scene(ok) == gsr.GSR_OK          # empty scene is valid
    assert gsr.gsr_validate_scene(gsr.gsr_scene(5, 0, None, None, None, None, None)) == gsr.GSR_EINVAL
    assert gsr.gsr_validate_scene(gsr.gsr_scene(-1, 0, None, None, None, None, None)) == gsr.GSR_EINVAL
    p = ctypes.c_void_p(64)
    assert gsr.gsr_validate_scene(gsr.gsr_scene(5, 3, p, p, p, p, p)) == gsr.GSR_OK
    assert gsr.gsr_validate_scene(gsr.gsr_scene(5, 4, p, p, p, p, p)) == gsr.GSR_EINVAL


@pytest.mark.parametrize("tile,batch,ok", [(16, 256, True), (8, 64, True), (8, 128, False), (32, 256, True),
                                            (12, 64, False), (16, 96, False)])
def test_validate_config_tiles(lib, tile, batch, ok):
    cfg = gsr.make_config(tile=tile, lds_batch=batch)
    assert (gsr.gsr_validate_config(cfg, _cam()) == gsr.GSR_OK) == ok


def test_validate_config_modes_and_thresholds(lib):
    for thr in (0, 1, 32, 64, 65):
        assert gsr.gsr_validate_config(gsr.make_config(reduce_threshold=thr)) == gsr.GSR_OK
    for thr in (-1, 66):
        assert gsr.gsr_validate_config(gsr.make_config(reduce_threshold=thr)) == gsr.GSR_EINVAL
    for mode in (0, 1, 2, 3, 4):
        assert gsr.gsr_validate_config(gsr.make_config(bwd_mode=mode)) == gsr.GSR_OK
    for mode in (-1, 5):
        assert gsr.gsr_validate_config(gsr.make_config(bwd_mode=mode)) == gsr.GSR_EINVAL
    assert gsr.gsr_validate_config(gsr.make_config(flags=1 << 10)) == gsr.GSR_EINVAL
    for mode in (0, 1, 2, 3, 4):   # both accumulator precisions exist for every mode
        assert gsr.gsr_validate_config(gsr.make_config(bwd_mode=mode, flags=gsr.GSR_FLAG_ACC_F32)) == gsr.GSR_OK
    # the compiler-reduced ablation has no counting build
    assert gsr.gsr_validate_config(gsr.make_config(bwd_mode=gsr.GSR_BWD_PLAIN_COMPILER_REDUCE,
                                                   flags=gsr.GSR_FLAG_DEBUG_COUNTERS)) == gsr.GSR_EINVAL
    assert gsr.gsr_validate_config(gsr.make_config(bwd_mode=gsr.GSR_BWD_PLAIN_ATOMIC,
                                                   flags=gsr.GSR_FLAG_DEBUG_COUNTERS)) == gsr.GSR_OK


def test_ctx_create_without_gpu_reports_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    out = ctypes.c_void_p()
    st = lib.gsr_ctx_create(ctypes.byref(out), 0, None)
    assert st != gsr.GSR_OK and not out.value


def test_server_scene_bytes(lib):
    # params, gradients and the two Adam moments: 4 x (3+3+4+1+3K) floats per Gaussian
    assert gsr.gsr_server_scene_bytes(1000, 3) == 1000 * 944
    assert gsr.gsr_server_scene_bytes(10, 0) == 10 * 4 * 14 * 4
    assert gsr.gsr_server_scene_bytes(-1, 0) == -1 and gsr.gsr_server_scene_bytes(5, 4) == -1


def test_server_rejects_bad_options_without_device(lib):
    # option checks run before any device call
    for bad in (dict(max_batch=0), dict(max_batch=17), dict(lanes=0), dict(lanes=5), dict(lr=0.0),
                dict(beta1=1.0), dict(eps=-1.0)):
        kw = dict(max_batch=4, lanes=2, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-15)
        kw.update(bad)
        opts = gsr.make_server_opts(1 << 30, **kw)
        with pytest.raises(gsr.GsrError):
            gsr.gsr_server_create(opts)
