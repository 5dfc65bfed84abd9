"""Pins of the oracle's binning and per-pixel composite (forward) against closed forms,
invariants and brute force."""
import math

import numpy as np

import oracle
from paper_2401_05345_amd import scenegen as sg


def sigmoid(x):
    return 1.0 / (1.0 + math.exp(-x))


def _scene(m, ls, q, op, dc):
    n = len(m)
    return sg.Scene(np.asarray(m, np.float32).reshape(n, 3), np.asarray(ls, np.float32).reshape(n, 3),
                    np.asarray(q, np.float32).reshape(n, 4), np.asarray(op, np.float32).reshape(n),
                    np.asarray(dc, np.float32).reshape(n, 1, 3), 0)


def _on_axis(depth):
    """World point on the optical axis: projects exactly onto the principal point."""
    return [0.0, 0.0, depth]


def test_single_gaussian_at_pixel_centre_closed_form():
    # alpha = min(0.99, sigmoid(omega)) and I = alpha rgb + (1 - alpha) bg at that pixel.
    for omega, bg in [(0.3, (0, 0, 0)), (-1.2, (0.2, 0.5, 0.9)), (6.0, (1, 0, 0.3))]:
        wl = sg.single_gaussian_at_pixel(9, 21, opacity_logit=omega)
        cam = wl.camera.with_bg(bg)
        rr = oracle.render(wl.scene, cam)
        alpha = min(0.99, sigmoid(np.float32(omega)))
        rgb = np.float32([0.7, 0.2, 0.4]).astype(np.float64) / (2 * math.sqrt(math.pi)) + 0.5
        bg32 = np.float32(bg).astype(np.float64)
        want = alpha * rgb + (1 - alpha) * bg32
        assert np.abs(rr.image[:, 21, 9] - want).max() < 1e-12
        assert abs(rr.T_final[21, 9] - (1 - alpha)) < 1e-15
        assert rr.n_contrib[21, 9] == 1


def test_two_gaussians_front_to_back_order():
    # The nearer Gaussian composites first regardless of index order:
    # I = a1 c1 + (1 - a1) a2 c2 + (1 - a1)(1 - a2) bg.
    cam = sg.single_gaussian_at_pixel(12, 7).camera.with_bg((0.1, 0.2, 0.3))
    far, near = _on_axis(4.0), _on_axis(2.0)
    sc = _scene([far, near], [[-3.5] * 3, [-3.0] * 3], [[1, 0, 0, 0]] * 2, [0.4, -0.7],
                [[0.9, 0.1, 0.3], [0.2, 0.8, 0.5]])
    rr = oracle.render(sc, cam)
    c = np.float32([[0.9, 0.1, 0.3], [0.2, 0.8, 0.5]]).astype(np.float64) / (2 * math.sqrt(math.pi)) + 0.5
    a_far, a_near = sigmoid(np.float32(0.4)), sigmoid(np.float32(-0.7))
    bg = np.float32([0.1, 0.2, 0.3]).astype(np.float64)
    want = a_near * c[1] + (1 - a_near) * a_far * c[0] + (1 - a_near) * (1 - a_far) * bg
    assert np.abs(rr.image[:, 7, 12] - want).max() < 1e-12
    assert rr.n_contrib[7, 12] == 2


def test_skipped_entries_count_in_n_contrib_and_early_stop():
    # Entry 1 (nearest) is far from the pixel (alpha < 1/255, skipped); entries 2 and 3 sit on
    # the pixel with alpha 0.99 (clamped) and 0.9; entry 4 (alpha 0.95) would push T below 1e-4:
    # the walk stops before it, so entry 5 (alpha 0.5, which alone would keep T >= 1e-4) is not
    # composited either. n_contrib = 3 (1-based, skipped entry counted), T_final = 0.01 * 0.1.
    px, py = 5, 5
    cam = sg.single_gaussian_at_pixel(px, py).camera
    off = [8.5 * 1.0 / cam.fx, 8.5 * 1.0 / cam.fy, 1.0]     # projects 8.5 px right and down
    pts = [off, _on_axis(2.0), _on_axis(3.0), _on_axis(4.0), _on_axis(5.0)]
    logit = lambda a: math.log(a / (1 - a))
    sc = _scene(pts, [[-3.2] * 3] * 5, [[1, 0, 0, 0]] * 5, [0.0, 8.0, logit(0.9), logit(0.95), 0.0],
                [[0.5, 0.5, 0.5], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0], [1.0, 1.0, 1.0]])
    rr = oracle.render(sc, cam)
    pos, ids = oracle.pixel_entries(rr, px, py)
    assert list(ids) == [1, 2] and list(pos) == [2, 3]
    assert rr.n_contrib[py, px] == 3
    a2 = sigmoid(np.float32(logit(0.9)))
    assert abs(rr.T_final[py, px] - 0.01 * (1 - a2)) < 1e-15


def test_weights_sum_to_one_and_transmittance_floor():
    # With every colour 1 and background 1 the image is exactly 1 (sum_k alpha_k T_k + T_final = 1);
    # with background 0 it is 1 - T_final. T_final >= 1e-4 everywhere.
    wl = sg.tiny_1k()
    sc = wl.scene
    ones = sg.Scene(sc.means3d, sc.log_scales, sc.quats, sc.opacity_logits,
                    np.zeros_like(sc.sh), 0)
    rr = oracle.render(ones, wl.camera.with_bg((1, 1, 1)))
    # rgb = 0.5 for a zero DC: the weights sum to one iff I = 0.5 (1 - T) + T.
    w = 1 - rr.T_final
    assert np.abs(rr.image - (0.5 * w + rr.T_final)[None]).max() < 1e-12
    rr0 = oracle.render(ones, wl.camera)
    assert np.abs(rr0.image - 0.5 * (1 - rr0.T_final)[None]).max() < 1e-12
    assert rr0.T_final.min() >= 1e-4
    assert (rr0.n_contrib > 0).mean() > 0.5


def test_image_in_unit_range():
    wl = sg.tiny_1k()
    # DC in U(0,1) gives rgb = f/(2 sqrt(pi)) + 0.5 in [0.5, 0.79]: a convex blend stays in [0,1].
    rr = oracle.render(wl.scene, wl.camera.with_bg((1.0, 0.0, 0.5)))
    assert (rr.proj.rgb >= 0).all() and (rr.proj.rgb <= 1.0).all()
    assert rr.image.min() >= 0.0 and rr.image.max() <= 1.0


def test_permutation_invariance():
    # Relabelling Gaussians (no depth ties) leaves the image bit-identical.
    wl = sg.tiny_1k()
    assert len(np.unique(oracle.project(wl.scene, wl.camera).depth_key)) == wl.scene.n
    perm = np.random.default_rng(11).permutation(wl.scene.n)
    rr = oracle.render(wl.scene, wl.camera)
    rp = oracle.render(wl.scene.subset(perm), wl.camera)
    assert np.array_equal(rr.image, rp.image)
    assert np.array_equal(rr.n_contrib, rp.n_contrib)


def test_depth_ties_ordered_by_index():
    # Two Gaussians at the same fp32 depth on one pixel: the lower index composites first.
    cam = sg.single_gaussian_at_pixel(8, 8).camera
    p = _on_axis(3.0)
    sc = _scene([p, p], [[-3.0] * 3] * 2, [[1, 0, 0, 0]] * 2, [0.5, 0.5], [[1, 0, 0], [0, 1, 0]])
    rr = oracle.render(sc, cam)
    pos, ids = oracle.pixel_entries(rr, 8, 8)
    assert list(ids) == [0, 1]
    assert rr.image[0, 8, 8] > rr.image[1, 8, 8]


def test_tile_lists_brute_force():
    # Exact equality with per-tile enumeration and Python's stable sort on (depth, index).
    for wl in (sg.tiny_1k(), sg.tiny_scene(9, 80, 50, 40, log_scale=(-1.8, 0.5))):
        pr = oracle.project(wl.scene, wl.camera, 16)
        tl = oracle.tile_lists(pr)
        gx, gy = pr.grid
        for t in range(gx * gy):
            tx, ty = t % gx, t // gx
            members = [g for g in range(pr.n) if pr.visible[g]
                       and pr.rect[g, 0] <= tx < pr.rect[g, 1] and pr.rect[g, 2] <= ty < pr.rect[g, 3]]
            members = sorted(members, key=lambda g: (float(pr.depth_key[g]), g))
            assert list(tl.ids[tl.tile_start[t]:tl.tile_start[t + 1]]) == members
        assert tl.tile_start[-1] == pr.tiles_touched.sum()


def test_tile_select_renders_only_selected_tiles():
    wl = sg.tiny_1k()
    full = oracle.render(wl.scene, wl.camera)
    sel = np.zeros(16, np.uint8)
    sel[[0, 5, 10]] = 1
    part = oracle.render(wl.scene, wl.camera, tile_select=sel)
    for t in range(16):
        ys, xs = slice((t // 4) * 16, (t // 4) * 16 + 16), slice((t % 4) * 16, (t % 4) * 16 + 16)
        if sel[t]:
            assert np.array_equal(part.image[:, ys, xs], full.image[:, ys, xs])
        else:
            assert (part.image[:, ys, xs] == 0).all()


def test_results_do_not_depend_on_the_thread_count():
    # The per-pixel loops run on OpenMP threads; the split must not change a single bit.
    wl = sg.tiny_scene(23, 400, 70, 45, sh_degree=1, log_scale=(-2.6, 0.5), half=0.7)
    cam = wl.camera.with_bg((0.2, 0.1, 0.3))
    r1 = oracle.render(wl.scene, cam, 16, threads=1)
    r4 = oracle.render(wl.scene, cam, 16, threads=4)
    for k in ("image", "T_final", "n_contrib", "margin", "signature"):
        assert np.array_equal(getattr(r1, k), getattr(r4, k)), k
    dl = np.random.default_rng(3).standard_normal((3, 45, 70))
    a1 = oracle.composite_backward(r1, dl, threads=1)
    a4 = oracle.composite_backward(r4, dl, threads=4)
    assert np.array_equal(a1, a4)
