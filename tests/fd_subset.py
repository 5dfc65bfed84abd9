"""The 50-Gaussian 32x32 crop of the 3M-Gaussian 1080p scene used for the
finite-difference checks (module name has no test_ prefix: not collected).

Gaussians are chosen among those the oracle's projection lists whose centre
falls in a 32x32 window around the image centre (a seeded draw); the crop
camera shifts the principal point by the window origin."""
from __future__ import annotations

import functools

import numpy as np

import oracle
from paper_2401_05345_amd import scenegen as sg

WINDOW = 32
COUNT = 50


@functools.lru_cache(maxsize=1)
def large_crop():
    wl = sg.large_3m()
    cam = wl.camera
    pr = oracle.project(wl.scene, cam)
    rng = np.random.default_rng(55)
    x0 = cam.width // 2 - WINDOW // 2
    y0 = cam.height // 2 - WINDOW // 2
    for _ in range(200):
        u, v = pr.mean2d[:, 0], pr.mean2d[:, 1]
        inside = np.nonzero(pr.visible & (u >= x0) & (u < x0 + WINDOW) & (v >= y0) & (v < y0 + WINDOW))[0]
        if inside.size >= COUNT:
            break
        x0 = int(rng.integers(0, cam.width - WINDOW))
        y0 = int(rng.integers(0, cam.height - WINDOW))
    pick = np.sort(rng.choice(inside, COUNT, replace=False))
    sub = wl.scene.subset(pick)
    ccam = cam.crop(x0, y0, WINDOW, WINDOW).with_bg((0.1, 0.2, 0.3))
    w = rng.standard_normal((3, WINDOW, WINDOW))
    return sub, ccam, w, (x0, y0), pick
