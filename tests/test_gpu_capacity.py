"""Capacity-mode re-render (no host synchronisation) and the graph-captured
training step.

* Re-rendering a state reproduces gsr_render's image, T_final, n_contrib and
  sorted lists bit for bit, also after the scene's parameters were changed in
  place (compared with a fresh render of the new parameters).
* A re-render whose pairs exceed the state's capacity reports the overflow and
  never writes past the buffers (the rest of the state stays usable).
* The captured step (re-render + loss gradient + batched backward), replayed
  with parameters changed between replays, equals the eager calls: images bit
  for bit, gradients to rel-L2 1e-5 (atomic order).
"""
import numpy as np
import pytest

from paper_2401_05345_amd import gsr
from paper_2401_05345_amd import scenegen as sg
from gpu_util import GpuScene, run_render, rel_l2, say

pytestmark = pytest.mark.gpu

NAMES = ["means3d", "log_scales", "quats", "opacity_logits", "sh"]
SPLIT = gsr.GSR_FLAG_LANE_SPLIT_ATOMICS


@pytest.fixture(scope="module")
def renderer(gsr):
    import torch
    r = gsr.Renderer(0)
    yield r
    torch.cuda.synchronize()
    r.close()


def _export_lists(r, st, gs):
    import torch
    P, over = gsr.gsr_fwd_sync(r.ctx, st)
    stats = gsr.gsr_fwd_stats(st)
    hw = gs.cam.width * gs.cam.height
    ex = dict(T_final=torch.zeros(hw, device="cuda:0"), n_contrib=torch.zeros(hw, dtype=torch.int32, device="cuda:0"),
              sorted_ids=torch.zeros(max(P, 1), dtype=torch.int32, device="cuda:0"),
              ranges=torch.zeros((stats.grid_x * stats.grid_y, 2), dtype=torch.int32, device="cuda:0"))
    gsr.gsr_fwd_export(r.ctx, st, **ex)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in ex.items()}
    out["sorted_ids"] = out["sorted_ids"][:P]
    return P, over, out


def test_rerender_reproduces_render(renderer):
    import torch
    say("[gpu] capacity-mode rerender")
    wl = sg.object_100k(n=20000, width=320, height=240)
    gs = GpuScene(wl.scene, wl.camera)
    cfg = gsr.make_config(16, 256, gsr.GSR_BWD_WAVE_REDUCE, 4, SPLIT)
    st, ref = run_render(renderer, gs, cfg)
    try:
        img = torch.full((3, gs.cam.height, gs.cam.width), float("nan"), device="cuda:0")
        for _ in range(2):
            gsr.gsr_rerender_batch(renderer.ctx, [st], [img], cfg)
            assert gsr.gsr_fwd_stats(st).n_pairs == -1
            P, over, out = _export_lists(renderer, st, gs)
            assert not over and P == int(ref["stats"].n_pairs)
            assert np.array_equal(img.cpu().numpy(), ref["image"])
            for k in ("T_final", "n_contrib", "sorted_ids", "ranges"):
                assert np.array_equal(out[k].reshape(-1), ref[k].reshape(-1)), k
        # parameters changed in place: the re-render equals a fresh render of the new values
        with torch.no_grad():
            gs.t["means3d"].add_(torch.randn_like(gs.t["means3d"]) * 0.01)
            gs.t["opacity_logits"].add_(0.3)
        gsr.gsr_rerender_batch(renderer.ctx, [st], [img], cfg)
        P, over, out = _export_lists(renderer, st, gs)
        s2, ref2 = run_render(renderer, gs, cfg)
        gsr.gsr_fwd_release(renderer.ctx, s2)
        assert not over and P == int(ref2["stats"].n_pairs)
        assert np.array_equal(img.cpu().numpy(), ref2["image"])
        for k in ("n_contrib", "sorted_ids", "ranges"):
            assert np.array_equal(out[k].reshape(-1), ref2[k].reshape(-1)), k
    finally:
        gsr.gsr_fwd_release(renderer.ctx, st)


def test_rerender_overflow_is_reported(renderer):
    import torch
    wl = sg.object_100k(n=5000, width=256, height=256)
    gs = GpuScene(wl.scene, wl.camera)
    cfg = gsr.make_config()
    st, ref = run_render(renderer, gs, cfg)
    try:
        P0 = int(ref["stats"].n_pairs)
        # Gaussians 20x larger touch many more tiles than the capacity (P0 * 1.25 + 4096) holds.
        with torch.no_grad():
            gs.t["log_scales"].add_(3.0)
        img = torch.zeros((3, gs.cam.height, gs.cam.width), device="cuda:0")
        gsr.gsr_rerender_batch(renderer.ctx, [st], [img], cfg)
        P, over = gsr.gsr_fwd_sync(renderer.ctx, st)
        assert over and P == P0 + P0 // 4 + 4096
        assert torch.isfinite(img).all()
        # the state still renders and differentiates (an incomplete image, no fault)
        g, gst = gs.grads()
        dl = torch.full_like(img, 1e-3)
        gsr.gsr_backward(renderer.ctx, st, dl, gst, 0, cfg)
        torch.cuda.synchronize()
        assert all(torch.isfinite(v).all() for v in g.values())
    finally:
        gsr.gsr_fwd_release(renderer.ctx, st)


@pytest.mark.parametrize("lam", [0.0, 0.2])
def test_graph_step_matches_eager(renderer, lam):
    import torch
    say(f"[gpu] graph-captured step, lambda={lam}")
    mv = sg.multi_view_small(seed=8)
    views = [(si, cam, tgt) for si, cam, tgt in mv.views if mv.scenes[si].n > 0][:5]
    gss = [GpuScene(mv.scenes[si], cam) for si, cam, _ in views]
    cfg = gsr.make_config(16, 256, gsr.GSR_BWD_WAVE_REDUCE, 4, SPLIT)
    imgs = [torch.zeros((3, g.cam.height, g.cam.width), device="cuda:0") for g in gss]
    tgts = [torch.from_numpy(t).cuda() for _, _, t in views]
    dls = [torch.zeros_like(i) for i in imgs]
    outs = [g.grads() for g in gss]
    states = gsr.gsr_render_batch(renderer.ctx, [g.scene for g in gss], [g.cam for g in gss], cfg, imgs)
    graph = None
    try:
        graph = gsr.gsr_graph_capture_step(renderer.ctx, states, imgs, tgts, dls, [o[1] for o in outs], lam, 0, cfg)
        for rep in range(3):
            with torch.no_grad():
                for g in gss:
                    g.t["means3d"].add_(torch.randn_like(g.t["means3d"]) * 0.003)
                    g.t["sh"].mul_(0.98)
            gsr.gsr_graph_launch(renderer.ctx, graph)
            torch.cuda.synchronize()
            got_img = [i.clone() for i in imgs]
            got = [{k: o[0][k].clone() for k in NAMES} for o in outs]
            # eager: fresh render, loss gradient, batched backward
            e_imgs = [torch.zeros_like(i) for i in imgs]
            e_dls = [torch.zeros_like(i) for i in imgs]
            e_outs = [g.grads() for g in gss]
            e_states = gsr.gsr_render_batch(renderer.ctx, [g.scene for g in gss], [g.cam for g in gss], cfg, e_imgs)
            for im, tg, d in zip(e_imgs, tgts, e_dls):
                if lam > 0:
                    gsr.gsr_l1_dssim_grad(renderer.ctx, im, tg, d, lam)
                else:
                    gsr.gsr_l1_grad(renderer.ctx, im, tg, d)
            gsr.gsr_backward_batch(renderer.ctx, e_states, e_dls, [o[1] for o in e_outs], 0, cfg)
            torch.cuda.synchronize()
            for st in e_states:
                gsr.gsr_fwd_release(renderer.ctx, st)
            for v in range(len(gss)):
                assert torch.equal(got_img[v], e_imgs[v]), (rep, v)
                assert gsr.gsr_fwd_sync(renderer.ctx, states[v])[1] is False
                for k in NAMES:
                    e = rel_l2(got[v][k].cpu().numpy(), e_outs[v][0][k].cpu().numpy())
                    assert e <= 1e-5, (rep, v, k, e)
    finally:
        if graph is not None:
            gsr.gsr_graph_destroy(renderer.ctx, graph)
        for st in states:
            gsr.gsr_fwd_release(renderer.ctx, st)
