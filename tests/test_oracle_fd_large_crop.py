"""Finite-difference pin of the oracle on the 50-Gaussian 32x32 crop of the
3M-Gaussian scene (SH degree 3, its scale and opacity distributions):
Richardson-extrapolated central differences, h and h/2, for every parameter
of ten Gaussians and a seeded sample of the rest. h = 1e-3 for scales,
opacities and SH; positions use h = 1e-5 and quaternions 1e-4, because these
splats span ~35 px at depth 4-6: a 1e-3 step moves a splat ~0.4 px or turns
its edge ~0.07 px, which flips some pixel's alpha cut (a decision change,
where no derivative exists, so that parameter is excluded)."""
import numpy as np
import pytest

import oracle
from paper_2401_05345_amd import scenegen as sg
from fd_subset import large_crop

pytestmark = pytest.mark.slow


def _signature(rr):
    p = rr.proj
    return (p.visible.tobytes(), p.rect.tobytes(), rr.lists.ids.tobytes(), rr.signature.tobytes(),
            rr.n_contrib.tobytes(), p.clamp_mask.tobytes(), p.frustum_clamp.tobytes())


def test_crop_backward_matches_finite_differences():
    sub, cam, w, _, _ = large_crop()
    base = [a.astype(np.float64) for a in sub.arrays()]
    mk = lambda arrs: sg.Scene(*arrs, sh_degree=3)
    rr = oracle.render(mk(base), cam)
    assert rr.n_contrib.max() > 0
    _, grads = oracle.backward(mk(base), rr, w)
    sig0 = _signature(rr)
    rng = np.random.default_rng(3)
    for ti, arr in enumerate(base):
        h = {0: 1e-5, 2: 1e-4}.get(ti, 1e-3)
        rows = set(rng.choice(arr.shape[0], 10, replace=False).tolist())
        flat_idx = [j for j in range(arr.size) if (j // (arr.size // arr.shape[0])) in rows]
        flat_idx += rng.choice(arr.size, min(40, arr.size), replace=False).tolist()
        fd, an = [], []
        for j in sorted(set(flat_idx)):
            vals, ok = [], True
            for step in (h, -h, h / 2, -h / 2):
                pert = [a.copy() for a in base]
                pert[ti].reshape(-1)[j] += step
                r2 = oracle.render(mk(pert), cam)
                if _signature(r2) != sig0:
                    ok = False
                    break
                vals.append(float((w * r2.image).sum()))
            if ok:
                fd.append((4 * (vals[2] - vals[3]) / h - (vals[0] - vals[1]) / (2 * h)) / 3)
                an.append(grads[ti].reshape(-1)[j])
        fd, an = np.array(fd), np.array(an)
        assert fd.size >= 0.5 * len(set(flat_idx)), ti
        scale = np.abs(an).max()
        assert scale > 0
        assert np.abs(fd - an).max() <= 1e-5 * scale, (ti, np.abs(fd - an).max(), scale)
