"""The allocation-free backward (gsr_backward_noalloc) against gsr_backward (collected last).

Both entry points run the same kernels; the allocation-free one keeps its
accumulator rows (and, on a state without a cached tile order, the order
table) in the library's fixed per-device scratch. Checked through the C ABI:

* two calls in a row, the second on a smaller view (the scratch keeps the
  first call's sums, so rows that must start at zero are really cleared),
  each equal to gsr_backward's gradients within rel-L2 1e-6 (fp64
  accumulators; only the order of fp64 atomic adds can differ);
* accumulate = 1 adds to the outputs like gsr_backward;
* a state above the stated maximum, and the debug counters, are refused on
  the host with GSR_EINVAL before anything is enqueued.
"""
import numpy as np
import pytest

from paper_2401_05345_amd import gsr
from paper_2401_05345_amd import scenegen as sg
from gpu_util import GpuScene, rel_l2, say, NAMES

pytestmark = pytest.mark.gpu

SPLIT = gsr.GSR_FLAG_LANE_SPLIT_ATOMICS


@pytest.fixture(scope="module")
def renderer(gsr):
    import torch
    r = gsr.Renderer(0)
    yield r
    torch.cuda.synchronize()
    r.close()


def _grads(gs, fill):
    g = {k: gs.torch.full_like(v, fill) for k, v in gs.t.items()}
    return g, gsr.make_grads(g["means3d"], g["log_scales"], g["quats"], g["opacity_logits"], g["sh"])


def _render(r, gs, cfg):
    torch = gs.torch
    img = torch.empty((3, gs.cam.height, gs.cam.width), device="cuda:0")
    return gsr.gsr_render(r.ctx, gs.scene, gs.cam, cfg, img), img


def _compare(gs, a, b, tol, label):
    for k in NAMES:
        x, y = a[k].cpu().numpy(), b[k].cpu().numpy()
        assert np.isfinite(x).all(), (label, k)
        e = rel_l2(x, y)
        say(f"[gpu] noalloc {label} {k}: rel-L2 {e:.2e}")
        assert e <= tol, (label, k, e)


@pytest.mark.parametrize("flags", [SPLIT, SPLIT | gsr.GSR_FLAG_ACC_F32])
def test_noalloc_backward_matches_backward_twice_then_smaller(renderer, flags):
    import torch
    big = sg.object_100k()
    small = sg.object_100k(seed=5, n=20_000, width=320, height=240)
    # fp32 accumulators add in the order the atomics land: same sums up to that order.
    tol = 1e-6 if not (flags & gsr.GSR_FLAG_ACC_F32) else 1e-4
    cfg = gsr.make_config(16, 256, gsr.GSR_BWD_WAVE_REDUCE, 2, flags)
    for label, wl in (("100k 800x800", big), ("20k 320x240", small)):
        say(f"[gpu] noalloc {label} flags={flags}")
        gs = GpuScene(wl.scene, wl.camera)
        st, img = _render(renderer, gs, cfg)
        try:
            dl = torch.from_numpy(np.random.default_rng(3).standard_normal(
                (3, gs.cam.height, gs.cam.width)).astype(np.float32) * 1e-3).cuda()
            # First on the fresh state (no tile order cached: the scratch holds it), then the
            # allocating entry point, then the allocation-free one again (cached order).
            g1, s1 = _grads(gs, float("nan"))
            gsr.gsr_backward_noalloc(renderer.ctx, st, dl, s1, 0, cfg)
            g0, s0 = _grads(gs, float("nan"))
            gsr.gsr_backward(renderer.ctx, st, dl, s0, 0, cfg)
            g2, s2 = _grads(gs, float("nan"))
            gsr.gsr_backward_noalloc(renderer.ctx, st, dl, s2, 0, cfg)
            torch.cuda.synchronize()
            _compare(gs, g1, g0, tol, label + " (scratch order)")
            _compare(gs, g2, g0, tol, label + " (cached order)")
            # accumulate = 1 adds onto what the outputs hold
            ga, sa = _grads(gs, 0.25)
            gsr.gsr_backward_noalloc(renderer.ctx, st, dl, sa, 1, cfg)
            torch.cuda.synchronize()
            for k in NAMES:
                want = g0[k].cpu().numpy() + np.float32(0.25)
                e = rel_l2(ga[k].cpu().numpy(), want)
                assert e <= max(tol, 1e-6), (label, "accumulate", k, e)
        finally:
            gsr.gsr_fwd_release(renderer.ctx, st)


def test_noalloc_refuses_what_it_cannot_hold(renderer):
    import torch
    n = gsr.GSR_NOALLOC_MAX_GAUSSIANS + 1
    wl = sg.object_100k(seed=6, n=n, width=64, height=64)
    gs = GpuScene(wl.scene, wl.camera)
    cfg = gsr.make_config(16, 256, gsr.GSR_BWD_WAVE_REDUCE, 2, SPLIT)
    st, _ = _render(renderer, gs, cfg)
    try:
        dl = torch.zeros((3, 64, 64), device="cuda:0")
        g, s = _grads(gs, 0.0)
        with pytest.raises(gsr.GsrError) as ei:
            gsr.gsr_backward_noalloc(renderer.ctx, st, dl, s, 0, cfg)
        assert ei.value.status == gsr.GSR_EINVAL and "exceed" in str(ei.value)
    finally:
        gsr.gsr_fwd_release(renderer.ctx, st)
    wl = sg.tiny_1k()
    gs = GpuScene(wl.scene, wl.camera)
    st, _ = _render(renderer, gs, cfg)
    try:
        dl = torch.zeros((3, 64, 64), device="cuda:0")
        g, s = _grads(gs, 0.0)
        with pytest.raises(gsr.GsrError) as ei:
            gsr.gsr_backward_noalloc(renderer.ctx, st, dl, s, 0,
                                     gsr.make_config(16, 256, gsr.GSR_BWD_WAVE_REDUCE, 2,
                                                     SPLIT | gsr.GSR_FLAG_DEBUG_COUNTERS))
        assert ei.value.status == gsr.GSR_EINVAL
        torch.cuda.synchronize()
    finally:
        gsr.gsr_fwd_release(renderer.ctx, st)
