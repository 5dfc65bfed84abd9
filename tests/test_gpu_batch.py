"""Batched render and backward: one composite launch over every (view, tile)
pair of up to 16 views of scenes of uneven size and resolution.

* Every view of a batch against the fp64 oracle, to the single-view
  tolerances (image rel-L2 <= 1e-5 away from tie pixels, n_contrib exact,
  gradients rel-L2 <= 1e-3).
* The batch against the same views rendered one at a time: image, T_final,
  n_contrib and the sorted lists are the same bits (per-pixel arithmetic does
  not depend on launch order); gradients agree to rel-L2 1e-5 (atomic order).
* Outputs shared by several views receive the sum of the views' gradients.
* The debug counters of a batch are the sums of the per-view counters.
* Argument errors are rejected before anything is enqueued.
"""
import numpy as np
import pytest

import oracle
from paper_2401_05345_amd import gsr
from paper_2401_05345_amd import scenegen as sg
from gpu_util import GpuScene, run_render, run_backward, tie_pixels, oracle_dl_dimage, rel_l2, say

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


@pytest.fixture(scope="module")
def small():
    mv = sg.multi_view_small()
    scenes = [s for s in mv.scenes]
    views = [(si, cam.with_bg((0.1 * (i % 3), 0.2, 0.05 * i)), tgt) for i, (si, cam, tgt) in enumerate(mv.views)]
    return scenes, views


def _gpu_views(scenes, views):
    return [GpuScene(scenes[si], cam) for si, cam, _ in views]


def _render_batch(r, gss, cfg):
    import torch
    imgs = [torch.full((3, g.cam.height, g.cam.width), float("nan"), device="cuda:0") for g in gss]
    states = gsr.gsr_render_batch(r.ctx, [g.scene for g in gss], [g.cam for g in gss], cfg, imgs)
    return states, imgs


def _export(r, g, st):
    import torch
    stats = gsr.gsr_fwd_stats(st)
    hw = g.cam.width * g.cam.height
    P = max(int(stats.n_pairs), 1)
    ex = dict(T_final=torch.zeros(hw, device="cuda:0"),
              n_contrib=torch.zeros(hw, dtype=torch.int32, device="cuda:0"),
              sorted_ids=torch.zeros(P, dtype=torch.int32, device="cuda:0"),
              ranges=torch.zeros((stats.grid_x * stats.grid_y, 2), dtype=torch.int32, device="cuda:0"))
    gsr.gsr_fwd_export(r.ctx, st, **ex)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in ex.items()}
    out["sorted_ids"] = out["sorted_ids"][: int(stats.n_pairs)]
    out["T_final"] = out["T_final"].reshape(g.cam.height, g.cam.width)
    out["n_contrib"] = out["n_contrib"].reshape(g.cam.height, g.cam.width)
    return out


def _backward_batch(r, gss, states, dls, cfg, shared=False, accumulate=0):
    import torch
    dts = [torch.from_numpy(np.ascontiguousarray(d, np.float32)).cuda() for d in dls]
    if shared:
        g, gs = gss[0].grads()
        outs = [(g, gs)] * len(gss)
    else:
        outs = [g.grads() for g in gss]
    gsr.gsr_backward_batch(r.ctx, states, dts, [o[1] for o in outs], accumulate, cfg)
    torch.cuda.synchronize()
    return [[o[0][k].cpu().numpy() for k in NAMES] for o in outs]


@pytest.mark.parametrize("flags", [SPLIT, SPLIT | gsr.GSR_FLAG_NO_TILE_ORDER])
def test_batch_matches_oracle(renderer, small, flags):
    scenes, views = small
    say(f"[gpu] batch of {len(views)} views vs oracle, flags={flags}")
    cfg = gsr.make_config(16, 256, gsr.GSR_BWD_WAVE_REDUCE, 4, flags)
    gss = _gpu_views(scenes, views)
    refs = [oracle.render(scenes[si], cam) for si, cam, _ in views]
    dls = [oracle_dl_dimage(rr, tgt, "l1") for rr, (_, _, tgt) in zip(refs, views)]
    states, imgs = _render_batch(renderer, gss, cfg)
    try:
        grads = _backward_batch(renderer, gss, states, dls, cfg)
        for i, (rr, g, st, img) in enumerate(zip(refs, gss, states, imgs)):
            out = _export(renderer, g, st)
            # Tie pixels need the projected radii and rectangles: take them from a single-view
            # render of the same view (the batch reproduces its bits, see the next test).
            s1, sout = run_render(renderer, g, cfg)
            gsr.gsr_fwd_release(renderer.ctx, s1)
            ties = tie_pixels(rr, sout)
            keep = ~ties
            assert ties.mean() < 0.02
            assert np.array_equal(out["n_contrib"][keep], rr.n_contrib[keep]), i
            e = rel_l2(img.cpu().numpy()[:, keep], rr.image[:, keep])
            assert e <= 1e-5, (i, e)
            _, gref = oracle.backward(scenes[views[i][0]], rr, dls[i].astype(np.float64))
            if g.n == 0:
                continue
            for name, a, b in zip(NAMES, grads[i], gref):
                err = rel_l2(a, b)
                assert err <= 1e-3, (i, name, err)
            say(f"[gpu] view {i}: n={g.n} {g.cam.width}x{g.cam.height} image {e:.1e}")
    finally:
        for st in states:
            gsr.gsr_fwd_release(renderer.ctx, st)


def test_batch_equals_single_views(renderer, small):
    scenes, views = small
    say("[gpu] batch vs single views")
    cfg = gsr.make_config(16, 256, gsr.GSR_BWD_WAVE_REDUCE, 4, SPLIT)
    gss = _gpu_views(scenes, views)
    dls = [np.random.default_rng(i).standard_normal((3, g.cam.height, g.cam.width)).astype(np.float32) * 1e-3
           for i, g in enumerate(gss)]
    states, imgs = _render_batch(renderer, gss, cfg)
    try:
        bgrads = _backward_batch(renderer, gss, states, dls, cfg)
        for i, (g, st, img) in enumerate(zip(gss, states, imgs)):
            bout = _export(renderer, g, st)
            s1, sout = run_render(renderer, g, cfg)
            try:
                assert np.array_equal(img.cpu().numpy(), sout["image"]), i
                assert np.array_equal(bout["T_final"], sout["T_final"]), i
                assert np.array_equal(bout["n_contrib"], sout["n_contrib"]), i
                assert np.array_equal(bout["ranges"], sout["ranges"]), i
                assert np.array_equal(bout["sorted_ids"], sout["sorted_ids"]), i
                sgrads, _, _ = run_backward(renderer, g, s1, dls[i], cfg)
                if g.n:
                    for name, a, b in zip(NAMES, bgrads[i], sgrads):
                        assert rel_l2(a, b) <= 1e-5, (i, name, rel_l2(a, b))
            finally:
                gsr.gsr_fwd_release(renderer.ctx, s1)
    finally:
        for st in states:
            gsr.gsr_fwd_release(renderer.ctx, st)


def test_shared_outputs_sum_views(renderer, small):
    # Two views of one scene writing one set of outputs get the sum of the views' gradients;
    # with accumulate=1 that sum is added to what the outputs held.
    import torch
    scenes, views = small
    pair = [v for v in views if v[0] == 2][:2]
    gss = _gpu_views(scenes, pair)
    gss[1].t = gss[0].t          # same device arrays for both views
    gss[1].scene = gss[0].scene
    cfg = gsr.make_config(16, 256, gsr.GSR_BWD_WAVE_REDUCE, 4, SPLIT)
    dls = [np.random.default_rng(7 + i).standard_normal((3, g.cam.height, g.cam.width)).astype(np.float32) * 1e-3
           for i, g in enumerate(gss)]
    states, _ = _render_batch(renderer, gss, cfg)
    try:
        summed = _backward_batch(renderer, gss, states, dls, cfg, shared=True)[0]
        sep = _backward_batch(renderer, gss, states, dls, cfg)
        for k, name in enumerate(NAMES):
            assert rel_l2(summed[k], sep[0][k] + sep[1][k]) <= 1e-5, name
        # accumulate=1: outputs start from ones
        g, gst = gss[0].grads()
        for v in g.values():
            v.fill_(1.0)
        dts = [torch.from_numpy(d).cuda() for d in dls]
        gsr.gsr_backward_batch(renderer.ctx, states, dts, [gst, gst], 1, cfg)
        torch.cuda.synchronize()
        for k, name in enumerate(NAMES):
            assert rel_l2(g[name].cpu().numpy(), 1.0 + sep[0][k] + sep[1][k]) <= 1e-5, name
    finally:
        for st in states:
            gsr.gsr_fwd_release(renderer.ctx, st)


def test_batch_counters_are_sums(renderer, small):
    scenes, views = small
    cfg = gsr.make_config(16, 256, gsr.GSR_BWD_WAVE_REDUCE, 8,
                          SPLIT | gsr.GSR_FLAG_DEBUG_COUNTERS)
    gss = _gpu_views(scenes, views)
    dls = [np.full((3, g.cam.height, g.cam.width), 1e-3, np.float32) for g in gss]
    states, _ = _render_batch(renderer, gss, cfg)
    try:
        _backward_batch(renderer, gss, states, dls, cfg)
        tot = gsr.gsr_bwd_counters(renderer.ctx, states[0])
        with pytest.raises(gsr.GsrError):
            gsr.gsr_bwd_counters(renderer.ctx, states[1])
        keys = ("evaluated", "active", "wave_entries", "reduced", "plain_lanes", "lane_atomics", "atomic_instrs",
                "visited")
        acc = dict.fromkeys(keys, 0)
        hist = np.zeros(65, np.int64)
        longest = 0
        for i, g in enumerate(gss):
            _backward_batch(renderer, [g], [states[i]], [dls[i]], cfg)
            c = gsr.gsr_bwd_counters(renderer.ctx, states[i])
            for k in keys:
                acc[k] += getattr(c, k)
            hist += np.array(c.hist[:], np.int64)
            longest = max(longest, c.max_wave_visits)
        for k in keys:
            assert getattr(tot, k) == acc[k], k
        assert tot.max_wave_visits == longest
        assert np.array_equal(np.array(tot.hist[:], np.int64), hist)
        assert tot.evaluated > 0
    finally:
        for st in states:
            gsr.gsr_fwd_release(renderer.ctx, st)


def test_batch_argument_errors(renderer, small):
    import torch
    scenes, views = small
    gss = _gpu_views(scenes, views[:3])
    cfg = gsr.make_config(16, 256, gsr.GSR_BWD_WAVE_REDUCE, 4, SPLIT)
    imgs = [torch.zeros((3, g.cam.height, g.cam.width), device="cuda:0") for g in gss]
    with pytest.raises(gsr.GsrError):
        gsr.gsr_render_batch(renderer.ctx, [], [], cfg, [])
    with pytest.raises(gsr.GsrError):
        gsr.gsr_render_batch(renderer.ctx, [gss[0].scene] * 17, [gss[0].cam] * 17, cfg, [imgs[0]] * 17)
    bad = gsr.make_camera(0, 10, 1.0, 1.0, 0.0, 0.0, views[0][1].world_to_cam)
    with pytest.raises(gsr.GsrError, match="view 1"):
        gsr.gsr_render_batch(renderer.ctx, [g.scene for g in gss], [gss[0].cam, bad, gss[2].cam], cfg, imgs)
    states, _ = _render_batch(renderer, gss, cfg)
    try:
        dls = [torch.zeros((3, g.cam.height, g.cam.width), device="cuda:0") for g in gss]
        outs = [g.grads() for g in gss]
        with pytest.raises(gsr.GsrError, match="share a state"):
            gsr.gsr_backward_batch(renderer.ctx, [states[0], states[0]], dls[:2], [outs[0][1], outs[1][1]])
        partial = gsr.make_grads(outs[0][0]["means3d"], outs[1][0]["log_scales"], outs[1][0]["quats"],
                                 outs[1][0]["opacity_logits"], outs[1][0]["sh"])
        with pytest.raises(gsr.GsrError, match="partly overlap"):
            gsr.gsr_backward_batch(renderer.ctx, states[:2], dls[:2], [outs[0][1], partial])
        with pytest.raises(gsr.GsrError, match="tile"):
            gsr.gsr_backward_batch(renderer.ctx, states, dls, [o[1] for o in outs], 0,
                                   gsr.make_config(8, 64, gsr.GSR_BWD_WAVE_REDUCE, 4, SPLIT))
    finally:
        for st in states:
            gsr.gsr_fwd_release(renderer.ctx, st)


def test_graph_replays_match_eager(renderer, small):
    # The captured batched backward, replayed several times with new dL/dimage values written
    # into the captured buffers and eager work (a single-view backward, torch fills) between
    # replays: every replay equals the eager batched backward of the same values.
    import torch
    scenes, views = small
    say("[gpu] graph-captured batched backward")
    cfg = gsr.make_config(16, 256, gsr.GSR_BWD_WAVE_REDUCE, 4, SPLIT)
    gss = _gpu_views(scenes, views)
    dls = [np.random.default_rng(20 + i).standard_normal((3, g.cam.height, g.cam.width)).astype(np.float32) * 1e-3
           for i, g in enumerate(gss)]
    states, _ = _render_batch(renderer, gss, cfg)
    graph = None
    try:
        eager = _backward_batch(renderer, gss, states, dls, cfg)
        dts = [torch.from_numpy(d).cuda() for d in dls]
        outs = [g.grads() for g in gss]
        graph = gsr.gsr_graph_capture_backward(renderer.ctx, states, dts, [o[1] for o in outs], 0, cfg)
        for rep in range(4):
            scale = float(rep + 1)
            for d, dn in zip(dts, dls):
                d.copy_(torch.from_numpy(dn * np.float32(scale)))
            for o in outs:
                for v in o[0].values():
                    v.fill_(float("nan"))
            gsr.gsr_graph_launch(renderer.ctx, graph)
            torch.cuda.synchronize()
            for i, (o, g) in enumerate(zip(outs, gss)):
                if g.n == 0:
                    continue
                for k, name in enumerate(NAMES):
                    e = rel_l2(o[0][name].cpu().numpy(), eager[i][k] * scale)
                    assert e <= 1e-5, (rep, i, name, e)
            run_backward(renderer, gss[0], states[0], dls[0], cfg)
            torch.cuda.synchronize()
    finally:
        if graph is not None:
            gsr.gsr_graph_destroy(renderer.ctx, graph)
        for st in states:
            gsr.gsr_fwd_release(renderer.ctx, st)


def test_autotune_picks_fastest_measured(renderer, small):
    scenes, views = small
    say("[gpu] autotune on the small batch")
    gss = _gpu_views(scenes, views)
    space = gsr.make_tune_space(reps=2, flags=SPLIT)
    best, entries = gsr.gsr_autotune(renderer.ctx, [g.scene for g in gss], [g.cam for g in gss], space)
    # (8,64), (16,64/128/256), (32,64/128/256) times nine thresholds
    assert len(entries) == 7 * 9
    seen = {(e.config.tile, e.config.lds_batch, e.config.reduce_threshold) for e in entries}
    assert len(seen) == 63
    tot = [e.render_ms + e.backward_ms for e in entries]
    k = int(np.argmin(tot))
    assert (best.tile, best.lds_batch, best.reduce_threshold) == \
        (entries[k].config.tile, entries[k].config.lds_batch, entries[k].config.reduce_threshold)
    assert best.bwd_mode == gsr.GSR_BWD_WAVE_REDUCE and best.flags == SPLIT
    assert all(e.render_ms > 0 and e.backward_ms > 0 for e in entries)
    say(f"[gpu] autotune best tile={best.tile} lds={best.lds_batch} thr={best.reduce_threshold} "
        f"{tot[k]:.3f} ms (worst {max(tot):.3f})")


def test_tuner_retunes_every_period(renderer, small):
    scenes, views = small
    gss = _gpu_views(scenes, views[:3])
    space = gsr.make_tune_space(tiles=(16,), batches=(256,), thresholds=(4, 32), reps=1, flags=SPLIT)
    t = gsr.gsr_tuner_create(space, 3)
    try:
        did = []
        for _ in range(7):
            cfg, d = gsr.gsr_tuner_next(renderer.ctx, t, [g.scene for g in gss], [g.cam for g in gss])
            did.append(d)
            assert cfg.tile == 16 and cfg.lds_batch == 256 and cfg.reduce_threshold in (4, 32)
        assert did == [True, False, False, True, False, False, True]
    finally:
        gsr.gsr_tuner_destroy(t)
