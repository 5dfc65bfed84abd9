"""Tile lists at scene sizes that take every path of the device scans and
radix sorts: a single scan block, the one-launch scan of up to 64k items in
one or two rounds, the two-level scan; 1024-item radix tiles below two
million items. For each size the exported lists must be the sorted order of
the pairs: the tile ranges partition [0, P), the entries increase strictly
in (tile, fp32 depth bits, id), every Gaussian appears exactly
tiles_touched times, and the visible count is the number of positive
radii."""
import numpy as np
import pytest

from paper_2401_05345_amd import gsr
from paper_2401_05345_amd import scenegen as sg
from gpu_util import GpuScene, run_render, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def renderer(gsr):
    import torch
    r = gsr.Renderer(0)
    yield r
    torch.cuda.synchronize()
    r.close()


@pytest.mark.parametrize("n,width,height", [(1, 64, 64), (2, 64, 64), (3000, 320, 240), (30_000, 640, 480),
                                            (50_000, 800, 600), (300_000, 1280, 720)])
def test_lists_are_sorted_at_every_size(renderer, n, width, height):
    say(f"[gpu] sort sizes n={n} {width}x{height}")
    wl = sg.object_100k(seed=11, n=n, width=width, height=height)
    _check_lists(renderer, wl.scene, wl.camera, n)


def test_lists_sorted_when_depths_share_their_high_bits(renderer):
    # Every depth in [4.5, 4.5001]: the visible depth keys differ only in their low bits, so the
    # upper passes of the depth sort copy instead of sorting.
    say("[gpu] sort with a narrow depth range")
    n = 20_000
    rng = np.random.default_rng(5)
    sc = sg.random_scene(rng, n, means="uniform", half=1.0, log_scale=(-3.5, 0.3), sh_degree=0)
    m = sc.means3d.copy()
    m[:, 2] = np.float32(0.5) + rng.uniform(0.0, 1e-4, n).astype(np.float32)
    sc = sg.Scene(m, sc.log_scales, sc.quats, sc.opacity_logits, sc.sh, 0)
    out = _check_lists(renderer, sc, sg.make_camera(640, 480, (0.0, 0.0, -4.0)), n)
    key = out["depth"].view(np.uint32)[out["radius"][:n] > 0]
    assert key.size > 1000 and int(key.min() ^ key.max()).bit_length() <= 16


def _check_lists(renderer, scene, camera, n):
    gs = GpuScene(scene, camera)
    st, out = run_render(renderer, gs, gsr.make_config())
    try:
        stats = out["stats"]
        P = int(stats.n_pairs)
        radius = out["radius"][:n]
        assert int(stats.n_visible) == int((radius > 0).sum())
        touched = out["tiles_touched"][:n].astype(np.int64)
        assert int(touched.sum()) == P
        if P == 0:
            return out
        ids = out["sorted_ids"].astype(np.int64)
        assert np.array_equal(np.bincount(ids, minlength=n), touched)
        rgs = out["ranges"].astype(np.int64)
        # every tile's range lies in [0, P) and is empty or ordered
        assert (rgs[:, 0] <= rgs[:, 1]).all() and rgs.min() >= 0 and rgs.max() <= P
        nonempty = rgs[:, 1] > rgs[:, 0]
        order = np.argsort(rgs[nonempty, 0])
        starts, ends = rgs[nonempty][order, 0], rgs[nonempty][order, 1]
        assert starts[0] == 0 and ends[-1] == P and np.array_equal(starts[1:], ends[:-1])
        tile_of = np.repeat(np.nonzero(nonempty)[0][order], ends - starts)
        key = out["depth"].view(np.uint32)[ids].astype(np.int64)
        if P > 1:
            step = np.stack([np.diff(tile_of), np.diff(key), np.diff(ids)], 1)
            first_nz = np.where(step[:, 0] != 0, step[:, 0], np.where(step[:, 1] != 0, step[:, 1], step[:, 2]))
            assert (first_nz > 0).all()
        return out
    finally:
        gsr.gsr_fwd_release(renderer.ctx, st)
