"""GPU edge cases and the reduce-or-atomic primitive's exact atomic-count model."""
import math

import numpy as np
import pytest

import oracle
from paper_2401_05345_amd import gsr
from paper_2401_05345_amd import scenegen as sg
from gpu_util import GpuScene, run_render, run_backward, rel_l2, say, oracle_dl_dimage

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def renderer(gsr):
    import torch
    r = gsr.Renderer(0)
    yield r
    torch.cuda.synchronize()
    r.close()


def _empty_scene(n=0, degree=0):
    return sg.Scene(np.zeros((n, 3), np.float32), np.zeros((n, 3), np.float32), np.zeros((n, 4), np.float32),
                    np.zeros(n, np.float32), np.zeros((n, (degree + 1) ** 2, 3), np.float32), degree)


def test_empty_scene_renders_background(renderer):
    say("[gpu] empty scene")
    cam = sg.make_camera(40, 24, (0, 0, -3), bg=(0.25, 0.5, 0.75))
    gs = GpuScene(_empty_scene(0), cam)
    cfg = gsr.make_config()
    st, out = run_render(renderer, gs, cfg)
    try:
        assert out["stats"].n_pairs == 0
        for c, b in enumerate((0.25, 0.5, 0.75)):
            assert (out["image"][c] == np.float32(b)).all()
        assert (out["T_final"] == 1).all() and (out["n_contrib"] == 0).all()
        run_backward(renderer, gs, st, np.ones((3, 24, 40), np.float32), cfg)
    finally:
        gsr.gsr_fwd_release(renderer.ctx, st)


def test_all_culled_gives_background_and_zero_gradients(renderer):
    say("[gpu] all culled")
    wl = sg.tiny_scene(3, 50, 32, 32, sh_degree=1)
    sc = wl.scene
    m = sc.means3d.copy()
    m[:, 2] = -6.0                 # all behind the camera
    sc = sg.Scene(m, sc.log_scales, sc.quats, sc.opacity_logits, sc.sh, 1)
    cam = wl.camera.with_bg((0.2, 0.2, 0.2))
    gs = GpuScene(sc, cam)
    cfg = gsr.make_config()
    st, out = run_render(renderer, gs, cfg)
    try:
        assert out["stats"].n_visible == 0 and out["stats"].n_pairs == 0
        assert (out["image"] == np.float32(0.2)).all()
        grads, acc, _ = run_backward(renderer, gs, st, np.ones((3, 32, 32), np.float32), cfg)
        for g in grads:
            assert (g == 0).all()
    finally:
        gsr.gsr_fwd_release(renderer.ctx, st)


def test_single_gaussian_closed_form(renderer):
    # alpha = min(0.99, sigmoid(omega)) at the pixel under the centre: I = alpha rgb + (1-alpha) bg.
    say("[gpu] single gaussian closed form")
    for omega in (0.3, 6.0):
        wl = sg.single_gaussian_at_pixel(9, 21, opacity_logit=omega)
        cam = wl.camera.with_bg((0.1, 0.2, 0.3))
        gs = GpuScene(wl.scene, cam)
        st, out = run_render(renderer, gs, gsr.make_config())
        gsr.gsr_fwd_release(renderer.ctx, st)
        a = min(0.99, 1 / (1 + math.exp(-float(np.float32(omega)))))
        rgb = np.float32([0.7, 0.2, 0.4]).astype(np.float64) / (2 * math.sqrt(math.pi)) + 0.5
        want = a * rgb + (1 - a) * np.float32([0.1, 0.2, 0.3]).astype(np.float64)
        assert np.abs(out["image"][:, 21, 9] - want).max() < 2e-7
        assert out["n_contrib"][21, 9] == 1


def test_large_image_one_row_of_partial_tiles(renderer):
    # 1080 rows at tile 16: the last tile row has 8 valid rows.
    say("[gpu] 1920x1080 partial tile row")
    rng = np.random.default_rng(4)
    sc = sg.random_scene(rng, 5000, means="clustered", half=2.0, log_scale=(-4.0, 0.5), sh_degree=0)
    cam = sg.make_camera(1920, 1080, (0, 0, -4))
    rr = oracle.render(sc, cam)
    gs = GpuScene(sc, cam)
    st, out = run_render(renderer, gs, gsr.make_config())
    try:
        keep = rr.margin >= 1e-4
        assert rel_l2(out["image"][:, keep], rr.image[:, keep]) <= 1e-5
        assert np.array_equal(out["n_contrib"][keep], rr.n_contrib[keep])
    finally:
        gsr.gsr_fwd_release(renderer.ctx, st)


def test_invalid_arguments_rejected_before_launch(renderer):
    say("[gpu] invalid args")
    wl = sg.tiny_1k()
    gs = GpuScene(wl.scene, wl.camera)
    bad = gsr.make_config(tile=12)
    with pytest.raises(gsr.GsrError) as e:
        run_render(renderer, gs, bad)
    assert e.value.status == gsr.GSR_EINVAL
    cam = gsr.make_camera(0, 10, 10.0, 10.0, 0, 0, np.eye(3, 4))
    import torch
    img = torch.zeros((3, 10, 10), device="cuda:0")
    with pytest.raises(gsr.GsrError):
        gsr.gsr_render(renderer.ctx, gs.scene, cam, gsr.make_config(), img)


def _model_atomics(active, mode, thr, split):
    """Exact number of atomic lane-operations the primitive must issue."""
    c = active.reshape(-1, 64).sum(1)
    if mode == gsr.GSR_BWD_PLAIN_ATOMIC:
        return int(9 * c.sum())
    t = max(thr, 1)
    red = (c >= t)
    per_reduced = 9
    return int(per_reduced * red.sum() + 9 * c[(c > 0) & ~red].sum())


@pytest.mark.parametrize("split", [0, 1])
def test_wave_reduce_primitive_sums_and_atomic_counts(renderer, split):
    import torch
    say(f"[gpu] wave reduce selftest split={split}")
    rng = np.random.default_rng(7)
    n_waves = 512
    # Active-lane densities from empty to full, so every threshold splits the waves differently.
    dens = rng.uniform(0, 1, size=n_waves)
    dens[:8] = 0.0
    dens[8:16] = 1.0
    active = (rng.uniform(size=(n_waves, 64)) < dens[:, None]).astype(np.uint8)
    vals = rng.standard_normal((n_waves, 64, 9)).astype(np.float32)
    want = (vals.astype(np.float64) * active[:, :, None]).sum((0, 1))
    dv = torch.from_numpy(vals).cuda()
    da = torch.from_numpy(active).cuda()
    sums = torch.zeros(9, device="cuda:0")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    scale = np.abs(vals).sum() / 9
    for mode in (gsr.GSR_BWD_PLAIN_ATOMIC, gsr.GSR_BWD_WAVE_REDUCE, gsr.GSR_BWD_SERIAL_REDUCE):
        for thr in (range(0, 66) if mode != gsr.GSR_BWD_PLAIN_ATOMIC else [0]):
            gsr.gsr_wave_reduce_selftest(renderer.ctx, dv, da, mode, thr, split, sums, cnt)
            torch.cuda.synchronize()
            got = sums.cpu().numpy().astype(np.float64)
            assert np.abs(got - want).max() <= 1e-5 * scale, (mode, thr)
            # A reduced wave issues nine lane-operations either way: lane 63 nine times, or nine lanes once.
            assert int(cnt.item()) == _model_atomics(active, mode, thr, split), (mode, thr)


def test_backward_counters_match_the_atomic_count_model(renderer):
    say("[gpu] counters model")
    wl = sg.object_100k(n=30000, width=400, height=300)
    cam = wl.camera
    rr = oracle.render(wl.scene, cam)
    gs = GpuScene(wl.scene, cam)
    keep = rr.margin >= 1e-4
    dl = np.random.default_rng(1).standard_normal((3, cam.height, cam.width)).astype(np.float32)
    for mode, thr, flags in [(gsr.GSR_BWD_PLAIN_ATOMIC, 0, 0), (gsr.GSR_BWD_WAVE_REDUCE, 1, 0),
                             (gsr.GSR_BWD_WAVE_REDUCE, 24, 0), (gsr.GSR_BWD_WAVE_REDUCE, 65, 0),
                             (gsr.GSR_BWD_WAVE_REDUCE, 16, gsr.GSR_FLAG_LANE_SPLIT_ATOMICS),
                             (gsr.GSR_BWD_SERIAL_REDUCE, 8, 0), (gsr.GSR_BWD_BLOCK_REDUCE, 1, 0),
                             (gsr.GSR_BWD_BLOCK_REDUCE, 24, 0)]:
        cfg = gsr.make_config(16, 256, mode, thr, gsr.GSR_FLAG_DEBUG_COUNTERS | flags)
        st, out = run_render(renderer, gs, cfg)
        try:
            run_backward(renderer, gs, st, dl, cfg)
            c = gsr.gsr_bwd_counters(renderer.ctx, st)
            hist = np.array(list(c.hist), np.int64)
            lanes = np.arange(65)
            # E and A against the oracle (exact where no pixel sits on a tie)
            if keep.all():
                assert c.evaluated == int(rr.n_contrib.sum())
                assert c.active == int(rr.n_used.sum())
            else:
                assert abs(int(c.evaluated) - int(rr.n_contrib.sum())) <= 64 * (~keep).sum()
            assert int(c.evaluated) == int(out["n_contrib"].astype(np.int64).sum())
            assert hist[0] == 0 and hist.sum() == c.wave_entries and (hist * lanes).sum() == c.active
            # every visited entry is a step of one wave's walk; the longest walk is one of them
            assert c.visited >= c.wave_entries and 0 < c.max_wave_visits <= c.visited
            # P_walk: every tile's block stages its list up to its deepest pixel's n_contrib
            nc = out["n_contrib"].astype(np.int64)
            gx, gy = -(-cam.width // 16), -(-cam.height // 16)
            pad = np.zeros((gy * 16, gx * 16), np.int64)
            pad[:cam.height, :cam.width] = nc
            assert c.walked == int(pad.reshape(gy, 16, gx, 16).max(axis=(1, 3)).sum())
            t = max(thr, 1)
            if mode == gsr.GSR_BWD_PLAIN_ATOMIC:
                assert c.reduced == 0 and c.plain_lanes == c.active
                assert c.lane_atomics == 9 * c.active and c.atomic_instrs == 9 * c.wave_entries
            elif mode == gsr.GSR_BWD_BLOCK_REDUCE:
                # reduced waves add into LDS; each (tile, Gaussian) touched by at least one of
                # them is flushed once: between a quarter of the reduced wave-entries (four
                # waves per 16x16 tile) and all of them.
                assert c.reduced == hist[t:].sum()
                assert c.plain_lanes == (hist[1:t] * lanes[1:t]).sum()
                flush = int(c.lane_atomics) - 9 * int(c.plain_lanes)
                assert flush % 9 == 0 and -(-int(c.reduced) // 4) <= flush // 9 <= int(c.reduced)
                flush_instrs = int(c.atomic_instrs) - 9 * int(c.wave_entries - c.reduced)
                assert -(-flush // 64) <= flush_instrs <= flush
            else:
                assert c.reduced == hist[t:].sum()
                assert c.plain_lanes == (hist[1:t] * lanes[1:t]).sum()
                per = 1 if (flags or mode == gsr.GSR_BWD_SERIAL_REDUCE) else 9
                assert c.lane_atomics == 9 * c.reduced + 9 * c.plain_lanes
                assert c.atomic_instrs == per * c.reduced + 9 * (c.wave_entries - c.reduced)
            say(f"[gpu] counters mode={mode} thr={thr}: E={c.evaluated} A={c.active} WE={c.wave_entries} "
                f"WR={c.reduced} A<={c.plain_lanes} lane_atomics={c.lane_atomics}")
        finally:
            gsr.gsr_fwd_release(renderer.ctx, st)


@pytest.mark.parametrize("degree", [0, 1, 2, 3])
def test_gradient_outputs_unaligned_and_accumulated(renderer, degree):
    # The per-Gaussian gradients leave as 16-byte stores when every output is 16-byte aligned
    # (SH rows of degrees 1 and 3 are whole 16-byte groups, stored group by group; degrees 0
    # and 2 go float by float), else one float at a time: both paths, and accumulate = 1 on
    # both, must write the same values bit for bit. 777 Gaussians leave a ragged last block.
    import torch
    say(f"[gpu] unaligned / accumulated gradient outputs, SH degree {degree}")
    wl = sg.tiny_scene(9, 777, 48, 40, sh_degree=degree, log_scale=(-2.4, 0.4), half=0.8)
    sc = wl.scene
    m = sc.means3d.copy()
    m[::5, 2] = -6.0                # every fifth Gaussian behind the camera: culled rows among visible ones
    wl.scene = sg.Scene(m, sc.log_scales, sc.quats, sc.opacity_logits, sc.sh, degree)
    cam = wl.camera.with_bg((0.1, 0.2, 0.3))
    gs = GpuScene(wl.scene, cam)
    cfg = gsr.make_config(16, 256, gsr.GSR_BWD_WAVE_REDUCE, 1)
    st, out = run_render(renderer, gs, cfg)
    try:
        rr = oracle.render(wl.scene, cam)
        dl = torch.from_numpy(oracle_dl_dimage(rr, wl.target, "l1")).cuda()
        gsr.gsr_backward_composite(renderer.ctx, st, dl, cfg)
        shapes = [v.shape for v in gs.t.values()]
        aligned = [torch.full(s, float("nan"), device="cuda:0") for s in shapes]
        gsr.gsr_backward_params(renderer.ctx, st, gsr.make_grads(*aligned), 0)
        bufs = [torch.full((int(np.prod(s)) + 1,), float("nan"), device="cuda:0") for s in shapes]
        shifted = [b[1:].view(s) for b, s in zip(bufs, shapes)]
        gsr.gsr_backward_params(renderer.ctx, st, gsr.make_grads(*shifted), 0)
        base = [torch.randn(s, device="cuda:0") for s in shapes]
        acc_a = [b.clone() for b in base]
        acc_u_bufs = [torch.zeros(int(np.prod(s)) + 1, device="cuda:0") for s in shapes]
        acc_u = [b[1:].view(s) for b, s in zip(acc_u_bufs, shapes)]
        for a, b in zip(acc_u, base):
            a.copy_(b)
        gsr.gsr_backward_params(renderer.ctx, st, gsr.make_grads(*acc_a), 1)
        gsr.gsr_backward_params(renderer.ctx, st, gsr.make_grads(*acc_u), 1)
        torch.cuda.synchronize()
        vis = torch.from_numpy(out["radius"] > 0).cuda()
        assert 0 < int(vis.sum()) < gs.n
        for a, u, b, ca, cu in zip(aligned, shifted, base, acc_a, acc_u):
            assert torch.isfinite(a).all()
            assert torch.equal(a.view(torch.int32), u.view(torch.int32))
            assert (a[~vis] == 0).all()
            assert torch.equal(ca, b + a) and torch.equal(cu, b + a)
        assert all(torch.isnan(b[0]) for b in bufs)   # nothing written before the shifted arrays
    finally:
        gsr.gsr_fwd_release(renderer.ctx, st)
