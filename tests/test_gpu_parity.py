"""GPU parity: the HIP path through the C ABI against the fp64 oracle.

Tolerances (stated for the path): relative L2 <= 1e-5 on the image and <= 1e-3
on each gradient tensor (atomic order is free). Integer results (radius, tile
counts, sort order, n_contrib) are compared exactly. Pixels whose per-pixel
decision sits within 1e-4 (relative) of its threshold, or whose tile is next to
a Gaussian whose radius/rectangle decision sits within 1e-3 px of a flip, admit
several correct results; they are excluded from the exact comparisons and
checked to be few.
"""
import numpy as np
import pytest

import oracle
from paper_2401_05345_amd import gsr
from paper_2401_05345_amd import scenegen as sg
from gpu_util import (GpuScene, run_render, run_backward, oracle_dl_dimage, rel_l2, say,
                      check_forward as _check_forward, check_grads as _check_grads, NAMES)

pytestmark = pytest.mark.gpu

@pytest.fixture(scope="module")
def renderer(gsr):
    import torch
    r = gsr.Renderer(0)
    yield r
    torch.cuda.synchronize()
    r.close()


def _workload_tiny():
    wl = sg.tiny_1k()
    return wl, wl.camera.with_bg((0.1, 0.3, 0.2))


@pytest.mark.parametrize("mode,thr,flags", [
    (gsr.GSR_BWD_PLAIN_ATOMIC, 0, 0),
    (gsr.GSR_BWD_WAVE_REDUCE, 0, 0),
    (gsr.GSR_BWD_WAVE_REDUCE, 32, 0),
    (gsr.GSR_BWD_WAVE_REDUCE, 64, 0),
    (gsr.GSR_BWD_WAVE_REDUCE, 65, 0),
    (gsr.GSR_BWD_WAVE_REDUCE, 8, gsr.GSR_FLAG_LANE_SPLIT_ATOMICS),
    (gsr.GSR_BWD_WAVE_REDUCE, 16, gsr.GSR_FLAG_XCD_REMAP),
    (gsr.GSR_BWD_SERIAL_REDUCE, 1, 0),
    (gsr.GSR_BWD_SERIAL_REDUCE, 24, 0),
    (gsr.GSR_BWD_BLOCK_REDUCE, 1, 0),
    (gsr.GSR_BWD_BLOCK_REDUCE, 32, 0),
    (gsr.GSR_BWD_PLAIN_ATOMIC, 0, gsr.GSR_FLAG_ACC_F32),
    (gsr.GSR_BWD_WAVE_REDUCE, 4, gsr.GSR_FLAG_ACC_F32 | gsr.GSR_FLAG_LANE_SPLIT_ATOMICS),
    (gsr.GSR_BWD_BLOCK_REDUCE, 1, gsr.GSR_FLAG_ACC_F32),
    (gsr.GSR_BWD_PLAIN_COMPILER_REDUCE, 0, 0),
    (gsr.GSR_BWD_PLAIN_COMPILER_REDUCE, 0, gsr.GSR_FLAG_ACC_F32),
])
def test_tiny_parity(renderer, mode, thr, flags):
    say(f"[gpu] tiny_1k parity mode={mode} thr={thr} flags={flags}")
    wl, cam = _workload_tiny()
    rr = oracle.render(wl.scene, cam)
    dl = oracle_dl_dimage(rr, wl.target, "l1")
    acc_ref, grads_ref = oracle.backward(wl.scene, rr, dl.astype(np.float64))
    gs = GpuScene(wl.scene, cam)
    cfg = gsr.make_config(16, 256, mode, thr, flags)
    st, out = run_render(renderer, gs, cfg)
    try:
        _check_forward(out, rr, 16)
        grads, acc, _ = run_backward(renderer, gs, st, dl, cfg)
        _check_grads(grads, acc, acc_ref, grads_ref)
    finally:
        gsr.gsr_fwd_release(renderer.ctx, st)


@pytest.mark.parametrize("tile,batch", [(8, 64), (16, 64), (16, 128), (32, 128), (32, 256)])
def test_tiles_and_batches_ragged_image(renderer, tile, batch):
    # 60x50 is not a multiple of any tile size: partial tiles have inactive lanes.
    say(f"[gpu] ragged 60x50 tile={tile} batch={batch}")
    wl = sg.tiny_scene(12, 300, 60, 50, sh_degree=2, log_scale=(-2.6, 0.5), half=0.7)
    cam = wl.camera.with_bg((0.3, 0.1, 0.6))
    rr = oracle.render(wl.scene, cam, tile)
    dl = oracle_dl_dimage(rr, wl.target, "l1")
    acc_ref, grads_ref = oracle.backward(wl.scene, rr, dl.astype(np.float64))
    gs = GpuScene(wl.scene, cam)
    for mode in (gsr.GSR_BWD_PLAIN_ATOMIC, gsr.GSR_BWD_WAVE_REDUCE, gsr.GSR_BWD_SERIAL_REDUCE,
                 gsr.GSR_BWD_BLOCK_REDUCE, gsr.GSR_BWD_PLAIN_COMPILER_REDUCE):
        cfg = gsr.make_config(tile, batch, mode, 24, 0)
        st, out = run_render(renderer, gs, cfg)
        try:
            _check_forward(out, rr, tile)
            grads, acc, _ = run_backward(renderer, gs, st, dl, cfg)
            _check_grads(grads, acc, acc_ref, grads_ref)
        finally:
            gsr.gsr_fwd_release(renderer.ctx, st)


def test_rotated_camera_parity(renderer):
    # A camera off the axes: the rotation's products round, so the fp32 depth key, the
    # lists and the colours exercise every term of the projection.
    say("[gpu] rotated camera parity")
    wl = sg.tiny_scene(44, 2000, 96, 80, sh_degree=3, log_scale=(-3.0, 0.5), eye=(1.3, -0.9, -2.6), half=0.8)
    cam = wl.camera.with_bg((0.05, 0.1, 0.15))
    rr = oracle.render(wl.scene, cam)
    dl = oracle_dl_dimage(rr, wl.target, "l1")
    acc_ref, grads_ref = oracle.backward(wl.scene, rr, dl.astype(np.float64))
    gs = GpuScene(wl.scene, cam)
    cfg = gsr.make_config(16, 256, gsr.GSR_BWD_WAVE_REDUCE, 4, gsr.GSR_FLAG_LANE_SPLIT_ATOMICS)
    st, out = run_render(renderer, gs, cfg)
    try:
        both = rr.proj.visible & (out["radius"] > 0)
        assert np.array_equal(out["depth"][both].view(np.uint32), rr.proj.depth_key[both].view(np.uint32))
        _check_forward(out, rr, 16)
        grads, acc, _ = run_backward(renderer, gs, st, dl, cfg)
        _check_grads(grads, acc, acc_ref, grads_ref)
    finally:
        gsr.gsr_fwd_release(renderer.ctx, st)


def test_object_100k_parity_and_modes(renderer):
    # 100k Gaussians, 800x800, SH degree 3, L1 + 0.2 D-SSIM against the perturbed scene's render.
    say("[gpu] object_100k parity")
    wl = sg.object_100k()
    cam = wl.camera
    rr = oracle.render(wl.scene, cam)
    target = oracle.render(wl.perturbed, cam).image
    dl = oracle_dl_dimage(rr, target, "l1_dssim")
    acc_ref, grads_ref = oracle.backward(wl.scene, rr, dl.astype(np.float64))
    gs = GpuScene(wl.scene, cam)
    cfg = gsr.make_config(16, 256, gsr.GSR_BWD_WAVE_REDUCE, 32, gsr.GSR_FLAG_DEBUG_COUNTERS)
    st, out = run_render(renderer, gs, cfg)
    try:
        img_err, ties = _check_forward(out, rr, 16)
        say(f"[gpu] object_100k image rel-L2 {img_err:.3e}, tie pixels {ties.sum()}")
        for mode, thr, flags in [(gsr.GSR_BWD_WAVE_REDUCE, 32, 0), (gsr.GSR_BWD_PLAIN_ATOMIC, 0, 0),
                                 (gsr.GSR_BWD_WAVE_REDUCE, 1, gsr.GSR_FLAG_LANE_SPLIT_ATOMICS),
                                 (gsr.GSR_BWD_SERIAL_REDUCE, 1, 0), (gsr.GSR_BWD_BLOCK_REDUCE, 1, 0),
                                 (gsr.GSR_BWD_WAVE_REDUCE, 1, gsr.GSR_FLAG_LANE_SPLIT_ATOMICS | gsr.GSR_FLAG_ACC_F32),
                                 (gsr.GSR_BWD_PLAIN_ATOMIC, 0, gsr.GSR_FLAG_ACC_F32),
                                 (gsr.GSR_BWD_PLAIN_COMPILER_REDUCE, 0, 0)]:
            grads, acc, _ = run_backward(renderer, gs, st, dl, gsr.make_config(16, 256, mode, thr, flags))
            errs = _check_grads(grads, acc, acc_ref, grads_ref)
            say(f"[gpu] object_100k mode={mode} thr={thr} grad rel-L2 {errs}")
    finally:
        gsr.gsr_fwd_release(renderer.ctx, st)


def test_forward_is_bitwise_deterministic(renderer):
    say("[gpu] determinism")
    wl = sg.object_100k(n=20000, width=320, height=240)
    gs = GpuScene(wl.scene, wl.camera)
    cfg = gsr.make_config()
    outs = []
    for _ in range(2):
        st, out = run_render(renderer, gs, cfg)
        gsr.gsr_fwd_release(renderer.ctx, st)
        outs.append(out)
    for k in ("image", "sorted_ids", "ranges", "T_final", "n_contrib", "radius"):
        assert np.array_equal(outs[0][k].view(np.uint8), outs[1][k].view(np.uint8)), k


def test_accumulate_adds(renderer):
    say("[gpu] accumulate")
    wl, cam = _workload_tiny()
    gs = GpuScene(wl.scene, cam)
    cfg = gsr.make_config(16, 256, gsr.GSR_BWD_WAVE_REDUCE, 32)
    st, out = run_render(renderer, gs, cfg)
    try:
        rr = oracle.render(wl.scene, cam)
        dl = oracle_dl_dimage(rr, wl.target, "l1")
        g1, _, held = run_backward(renderer, gs, st, dl, cfg)
        g2, _, _ = run_backward(renderer, gs, st, dl, cfg, accumulate=1, grads=held)
        for a, b in zip(g1, g2):
            assert rel_l2(b, 2 * a) < 1e-4      # two backwards differ only by atomic summation order
    finally:
        gsr.gsr_fwd_release(renderer.ctx, st)
