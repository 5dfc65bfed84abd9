"""The seeded input generators: identical seeds give identical bytes, different
seeds differ, and the workloads have the documented shapes and draws."""
import hashlib

import numpy as np

from paper_2401_05345_amd import scenegen as sg


def _digest(arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def test_same_seed_same_bytes():
    a, b = sg.tiny_1k(), sg.tiny_1k()
    assert _digest(a.scene.arrays() + (a.target, a.camera.world_to_cam)) == \
        _digest(b.scene.arrays() + (b.target, b.camera.world_to_cam))
    m1, m2 = sg.multi_view_small(), sg.multi_view_small()
    assert _digest([x for s in m1.scenes for x in s.arrays()]) == _digest([x for s in m2.scenes for x in s.arrays()])
    assert all(np.array_equal(v1[1].world_to_cam, v2[1].world_to_cam) and np.array_equal(v1[2], v2[2])
               for v1, v2 in zip(m1.views, m2.views))
    r1, r2 = sg.serving_requests(3, 10, 50, 200.0), sg.serving_requests(3, 10, 50, 200.0)
    assert [(t, s, seed) for t, s, _, seed in r1] == [(t, s, seed) for t, s, _, seed in r2]


def test_different_seeds_differ():
    assert _digest(sg.tiny_1k(1).scene.arrays()) != _digest(sg.tiny_1k(2).scene.arrays())


def test_workload_shapes():
    wl = sg.tiny_1k()
    assert wl.scene.n == 1000 and wl.scene.sh.shape == (1000, 1, 3) and wl.target.shape == (3, 64, 64)
    assert np.allclose(np.linalg.norm(wl.scene.quats, axis=1), 1.0, atol=1e-6)
    assert wl.scene.sh[:, 0].min() >= 0.0 and wl.scene.sh[:, 0].max() < 1.0
    mv = sg.multi_view_small()
    assert [s.n for s in mv.scenes] == [600, 2500, 6000, 0] and len(mv.views) == 8
    for si, cam, tgt in mv.views:
        assert tgt.shape == (3, cam.height, cam.width)
        R = cam.world_to_cam[:, :3].astype(np.float64)
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-5)
        eye = -R.T @ cam.world_to_cam[:, 3]
        assert abs(np.linalg.norm(eye) - 4.0) < 1e-4        # eyes on the r = 4 sphere


def test_poisson_arrivals():
    reqs = sg.serving_requests(11, 10, 4000, 400.0)
    t = np.array([r[0] for r in reqs])
    assert np.all(np.diff(t) > 0)
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert abs(gaps.mean() - 1 / 400.0) < 0.1 / 400.0     # mean gap 1/rate
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.1       # exponential: coefficient of variation 1
    scenes = np.bincount([r[1] for r in reqs], minlength=10)
    assert scenes.min() > 300                               # uniform over the ten scenes
