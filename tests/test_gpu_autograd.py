"""torch.autograd.Function over the HIP render/backward.

* The 50-Gaussian 32x32 crop of the 3M-Gaussian scene: image and gradients
  against the fp64 oracle (whose own finite differences pin it in
  test_oracle_fd_large_crop.py), and fp32 central differences of the GPU
  forward against the GPU gradient for the SH and opacity parameters.
* The full 3M-Gaussian 1920x1080 view through autograd with an L1 loss
  computed by torch: the gradients equal those of the direct C-ABI backward
  given the same dL/dimage.
"""
import numpy as np
import pytest

import oracle
from paper_2401_05345_amd import gsr
from paper_2401_05345_amd import scenegen as sg
from paper_2401_05345_amd.autograd import rasterize
from fd_subset import large_crop
from gpu_util import rel_l2, say, GpuScene, run_render, run_backward

pytestmark = pytest.mark.gpu

NAMES = ["means3d", "log_scales", "quats", "opacity_logits", "sh"]


@pytest.fixture(scope="module")
def renderer(gsr):
    import torch
    r = gsr.Renderer(0)
    yield r
    torch.cuda.synchronize()
    r.close()


def _params(scene, requires_grad=True):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda().requires_grad_(requires_grad)
            for a in scene.arrays()]


def _cam(c):
    return gsr.make_camera(c.width, c.height, c.fx, c.fy, c.cx, c.cy, c.world_to_cam, c.znear, c.bg)


def test_autograd_on_large_crop_matches_oracle(renderer):
    import torch
    say("[gpu] autograd crop")
    sub, cam, w, _, _ = large_crop()
    w32 = w.astype(np.float32)
    params = _params(sub)
    img = rasterize(*params, renderer=renderer, camera=_cam(cam))
    loss = (img * torch.from_numpy(w32).cuda()).sum()
    loss.backward()
    rr = oracle.render(sub, cam)
    _, ref = oracle.backward(sub, rr, w32.astype(np.float64))
    keep = rr.margin >= 1e-4
    assert rel_l2(img.detach().cpu().numpy()[:, keep], rr.image[:, keep]) <= 1e-5
    for name, p, r in zip(NAMES, params, ref):
        e = rel_l2(p.grad.cpu().numpy(), r)
        say(f"[gpu] crop {name} rel-L2 {e:.2e}")
        assert e <= 1e-3, (name, e)


def test_autograd_fp32_finite_differences(renderer):
    # Central differences of the GPU forward (fp32 image, the weighted sum taken in fp64) against
    # the GPU gradient, for all five tensors. SH enters linearly (away from the colour clamp) and
    # opacity smoothly; the geometry (means, log-scales, quaternions) is smooth too except where a
    # step moves a splat across a tile edge or an alpha threshold, which a small step rarely does
    # (the median over the sampled entries is the bound, the worst entry is reported).
    import torch
    say("[gpu] autograd fp32 FD")
    sub, cam, w, _, _ = large_crop()
    wt = torch.from_numpy(w.astype(np.float32)).cuda().double()
    params = _params(sub)
    (rasterize(*params, renderer=renderer, camera=_cam(cam)) * wt.float()).sum().backward()
    rng = np.random.default_rng(9)
    for ti, h in ((4, 1e-2), (3, 1e-2), (0, 1e-3), (1, 1e-3), (2, 1e-3)):
        grad = params[ti].grad.cpu().numpy().reshape(-1)
        fd, an = [], []
        for j in rng.choice(grad.size, 24, replace=False):
            vals = []
            for s in (h, -h):
                q = [p.detach().clone() for p in params]
                q[ti].view(-1)[j] += s
                with torch.no_grad():
                    img = rasterize(*q, renderer=renderer, camera=_cam(cam))
                    vals.append(float((img.double() * wt).sum()))
            fd.append((vals[0] - vals[1]) / (2 * h))
            an.append(grad[j])
        fd, an = np.array(fd), np.array(an)
        err = np.abs(fd - an) / (np.abs(an).max() + 1e-12)
        say(f"[gpu] fp32 FD tensor {NAMES[ti]}: median rel {np.median(err):.2e}, max {err.max():.2e}")
        assert np.median(err) <= 1e-2, (NAMES[ti], np.median(err))


def test_autograd_full_large_view_equals_direct_backward(renderer):
    import torch
    say("[gpu] autograd full 3M view")
    wl = sg.large_3m()
    cfg = gsr.make_config(16, 256, gsr.GSR_BWD_WAVE_REDUCE, 4, gsr.GSR_FLAG_LANE_SPLIT_ATOMICS)
    params = _params(wl.scene)
    target = torch.from_numpy(wl.target).cuda()
    img = rasterize(*params, renderer=renderer, camera=_cam(wl.camera), config=cfg)
    img.retain_grad()
    loss = (img - target).abs().mean()
    loss.backward()
    dl = img.grad.detach().cpu().numpy()
    gs = GpuScene(wl.scene, wl.camera)
    st, out = run_render(renderer, gs, cfg)
    try:
        assert np.array_equal(out["image"], img.detach().cpu().numpy())   # same forward, bit for bit
        grads, _, _ = run_backward(renderer, gs, st, dl, cfg)
        again, _, _ = run_backward(renderer, gs, st, dl, cfg)
        # fp32 accumulators (the paper's setting): the order of the atomic adds shows
        cfg32 = gsr.make_config(16, 256, gsr.GSR_BWD_WAVE_REDUCE, 4,
                                gsr.GSR_FLAG_LANE_SPLIT_ATOMICS | gsr.GSR_FLAG_ACC_F32)
        d32a, _, _ = run_backward(renderer, gs, st, dl, cfg32)
        d32b, _, _ = run_backward(renderer, gs, st, dl, cfg32)
    finally:
        gsr.gsr_fwd_release(renderer.ctx, st)
    # fp64 accumulators (the default): autograd and two direct runs give the same sums (their
    # parity with the oracle over the whole frame is test_gpu_large.py's).
    # fp32 accumulators (the paper's setting) are NOT within the 1e-3 gradient tolerance on this
    # view: the screen-filling splats collect ~1e4 wave sums with heavy cancellation, and the
    # order in which fp32 atomics add them moves the quaternion and scale gradients by ~1e-3
    # from run to run. The bound below is no parity claim; it only checks that the fp32 sums are
    # the same sums up to that ordering noise (a wrong term would be far above it).
    for name, p, g, h, a32, b32 in zip(NAMES, params, grads, again, d32a, d32b):
        e, floor64 = rel_l2(p.grad.cpu().numpy(), g), rel_l2(h, g)
        floor32, e32 = rel_l2(b32, a32), rel_l2(a32, g)
        say(f"[gpu] full 3M {name}: autograd vs direct {e:.2e}, direct runs {floor64:.2e} (fp64 acc); "
            f"fp32 acc runs {floor32:.2e}, fp32 vs fp64 {e32:.2e} (fp32 accumulators: outside parity here)")
        assert e <= 1e-5 and floor64 <= 1e-5, (name, e, floor64)
        ordering_noise_bound = 1e-2
        assert e32 <= ordering_noise_bound, (name, e32, floor32)
