"""fp64 oracle, per-Gaussian part: projection, EWA splat covariance and colour,
and the chain rule from the nine per-Gaussian accumulators back to the raw
parameters.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU
baseline leg of the benchmark, never by the product path. It shares no code
with the HIP path.

The paper (Background, "Differentiable Rendering for Rasterization
Pipelines") names 3D Gaussian Splatting as the renderer it instruments but
does not restate its math; this module follows the published 3DGS method:
sigmoid opacity, exponential scales, a normalised quaternion, the 3D
covariance R S S^T R^T, the EWA projection J W Sigma W^T J^T with a 0.3 px
low-pass, a 3-sigma radius and view-dependent colour from real spherical
harmonics up to degree 3 with a +0.5 offset, clamped at zero.

Every continuous value is computed in float64 with torch on the CPU. The
step the paper calls "gradients for all the parameters" (the last stage of
its rasterisation pipeline figure) is taken with torch.autograd through the
same float64 forward function: the definition of the derivative, evaluated
by a library primitive, with nothing hand-derived.

Discrete decisions: the depth sort key and the near-plane cull are taken on
the fp32 depth computed as ((R20*mx + R21*my) + R22*mz) + t2, one correctly
rounded fp32 operation at a time (the precision the kernel takes them in;
fp32 products and sums are exactly reproducible). Radius, tile rectangle and
the per-pixel alpha/transmittance decisions go through exp/sqrt and are
taken in float64; their distance to the decision threshold is reported so a
comparison can tell ties (several valid results) from errors.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

DT = torch.float64
LOWPASS = 0.3
GUARD = 0.15   # the Jacobian's x/z, y/z are held within the image extended by 15 % of its size per side


def sh_constants():
    """Normalisation constants of the real spherical harmonics, l <= 3, from their closed forms."""
    pi = math.pi
    return {
        "c0": math.sqrt(1.0 / (4.0 * pi)),
        "c1": math.sqrt(3.0 / (4.0 * pi)),
        "c2_xy": 0.5 * math.sqrt(15.0 / pi),
        "c2_zz": 0.25 * math.sqrt(5.0 / pi),
        "c2_xx_yy": 0.25 * math.sqrt(15.0 / pi),
        "c3_a": 0.25 * math.sqrt(35.0 / (2.0 * pi)),
        "c3_xyz": 0.5 * math.sqrt(105.0 / pi),
        "c3_b": 0.25 * math.sqrt(21.0 / (2.0 * pi)),
        "c3_z": 0.25 * math.sqrt(7.0 / pi),
        "c3_zxy": 0.25 * math.sqrt(105.0 / pi),
    }


def sh_basis(d: torch.Tensor, degree: int) -> torch.Tensor:
    """Real SH basis Y_k(d), k = l*l + l + m, for unit directions d [M,3] -> [M,K].

    Sign convention: the l=1 terms are proportional to (-y, z, -x)
    (Condon-Shortley phase), and likewise for l=2,3.
    """
    c = sh_constants()
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    out = [torch.full_like(x, c["c0"])]
    if degree >= 1:
        out += [-c["c1"] * y, c["c1"] * z, -c["c1"] * x]
    if degree >= 2:
        xx, yy, zz = x * x, y * y, z * z
        out += [c["c2_xy"] * x * y, -c["c2_xy"] * y * z, c["c2_zz"] * (2 * zz - xx - yy),
                -c["c2_xy"] * x * z, c["c2_xx_yy"] * (xx - yy)]
    if degree >= 3:
        out += [-c["c3_a"] * y * (3 * xx - yy), c["c3_xyz"] * x * y * z,
                -c["c3_b"] * y * (4 * zz - xx - yy), c["c3_z"] * z * (2 * zz - 3 * xx - 3 * yy),
                -c["c3_b"] * x * (4 * zz - xx - yy), c["c3_zxy"] * z * (xx - yy),
                -c["c3_a"] * x * (xx - 3 * yy)]
    return torch.stack(out, dim=1)


def quat_to_rot(q: torch.Tensor) -> torch.Tensor:
    """Rotation matrix of the unit quaternion q = (w, x, y, z) (Hamilton convention) [M,4] -> [M,3,3]."""
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    r = torch.stack([
        1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
        2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
        2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y),
    ], dim=1)
    return r.reshape(-1, 3, 3)


def covariance3d(log_scales: torch.Tensor, quats: torch.Tensor) -> torch.Tensor:
    """Sigma = R S S^T R^T with S = diag(exp(s)) and R the rotation of q/|q| [M,3,3]."""
    s = torch.exp(log_scales)
    R = quat_to_rot(quats / torch.linalg.norm(quats, dim=1, keepdim=True))
    M = R * s[:, None, :]                      # R diag(s)
    return M @ M.transpose(1, 2)


def depth_key_f32(means3d: np.ndarray, world_to_cam: np.ndarray) -> np.ndarray:
    """fp32 camera-space depth ((R20*mx + R21*my) + R22*mz) + t2, one fp32 op at a time."""
    m = np.asarray(means3d, np.float32)
    w = np.asarray(world_to_cam, np.float32)
    r20, r21, r22, t2 = w[2, 0], w[2, 1], w[2, 2], w[2, 3]
    s = np.multiply(r20, m[:, 0], dtype=np.float32)
    s = np.add(s, np.multiply(r21, m[:, 1], dtype=np.float32), dtype=np.float32)
    s = np.add(s, np.multiply(r22, m[:, 2], dtype=np.float32), dtype=np.float32)
    return np.add(s, t2, dtype=np.float32)


def splat_params(means, log_scales, quats, opacity_logits, sh, cam):
    """Differentiable per-Gaussian forward (float64 tensors) for Gaussians in front of the camera.

    Returns u, v, (a, b, c) of the 2D covariance, conic (A, B, C), opacity o,
    rgb (clamped) and rgb_raw.
    """
    W = torch.tensor(np.asarray(cam.world_to_cam, np.float32).astype(np.float64), dtype=DT)
    Rc, tc = W[:, :3], W[:, 3]
    fx, fy = float(np.float32(cam.fx)), float(np.float32(cam.fy))
    cx, cy = float(np.float32(cam.cx)), float(np.float32(cam.cy))

    t = means @ Rc.T + tc
    tx, ty, tz = t[:, 0], t[:, 1], t[:, 2]

    o = torch.sigmoid(opacity_logits)
    Sigma = covariance3d(log_scales, quats)

    # Guard band: with the principal point at the centre this is 3DGS's +-1.3 * half-extent / focal.
    lox, hix = (-cx - GUARD * cam.width) / fx, (cam.width - cx + GUARD * cam.width) / fx
    loy, hiy = (-cy - GUARD * cam.height) / fy, (cam.height - cy + GUARD * cam.height) / fy
    xc = torch.clamp(tx / tz, lox, hix) * tz
    yc = torch.clamp(ty / tz, loy, hiy) * tz
    zeros = torch.zeros_like(tz)
    J = torch.stack([
        torch.stack([fx / tz, zeros, -fx * xc / (tz * tz)], dim=1),
        torch.stack([zeros, fy / tz, -fy * yc / (tz * tz)], dim=1),
    ], dim=1)                                   # [M,2,3]
    Tm = J @ Rc                                 # [M,2,3]
    S2 = Tm @ Sigma @ Tm.transpose(1, 2)
    a = S2[:, 0, 0] + LOWPASS
    b = S2[:, 0, 1]
    c = S2[:, 1, 1] + LOWPASS
    det = a * c - b * b
    A, B, C = c / det, -b / det, a / det

    u = fx * tx / tz + cx
    v = fy * ty / tz + cy

    cam_centre = -(Rc.T @ tc)
    dvec = means - cam_centre
    dirs = dvec / torch.linalg.norm(dvec, dim=1, keepdim=True)
    Y = sh_basis(dirs, int(round(math.sqrt(sh.shape[1]))) - 1)
    rgb_raw = torch.einsum("mk,mkc->mc", Y, sh) + 0.5
    rgb = torch.clamp(rgb_raw, min=0.0)
    fcl = (((tx / tz) < lox) | ((tx / tz) > hix)).to(torch.uint8) + 2 * (((ty / tz) < loy) | ((ty / tz) > hiy)).to(torch.uint8)
    return dict(u=u, v=v, a=a, b=b, c=c, det=det, A=A, B=B, C=C, o=o, rgb=rgb, rgb_raw=rgb_raw,
                frustum_clamp=fcl)


@dataclass
class Projected:
    n: int
    visible: np.ndarray        # bool [n]
    depth_key: np.ndarray      # fp32 [n]
    mean2d: np.ndarray         # f64 [n,2]
    conic: np.ndarray          # f64 [n,3]
    opacity: np.ndarray        # f64 [n]
    rgb: np.ndarray            # f64 [n,3]
    cov2d: np.ndarray          # f64 [n,3] (a, b, c)
    radius: np.ndarray         # int64 [n], 0 when culled
    rect: np.ndarray           # int64 [n,4] x_lo, x_hi, y_lo, y_hi
    tiles_touched: np.ndarray  # int64 [n]
    clamp_mask: np.ndarray     # uint8 [n], bit c set when channel c was clamped at 0
    geom_margin: np.ndarray    # f64 [n], px distance of radius/rect decisions to a flip
    frustum_clamp: np.ndarray  # uint8 [n], bit0/bit1 when x/y of t/t_z was clamped to the 1.3 guard band
    grid: tuple


def _to64(a):
    """float32 inputs are upcast exactly; float64 inputs (finite differences) pass through."""
    a = np.asarray(a)
    if a.dtype != np.float64:
        a = a.astype(np.float32).astype(np.float64)
    return torch.tensor(a, dtype=DT)


def project(scene, cam, tile: int = 16) -> Projected:
    """Per-Gaussian forward of the renderer: everything the per-pixel pass needs."""
    n = scene.n
    gx = (cam.width + tile - 1) // tile
    gy = (cam.height + tile - 1) // tile
    dk = depth_key_f32(scene.means3d, cam.world_to_cam) if n else np.zeros(0, np.float32)
    front = dk > np.float32(cam.znear)
    idx = np.nonzero(front)[0]

    out = Projected(n, np.zeros(n, bool), dk, np.zeros((n, 2)), np.zeros((n, 3)), np.zeros(n),
                    np.zeros((n, 3)), np.zeros((n, 3)), np.zeros(n, np.int64), np.zeros((n, 4), np.int64),
                    np.zeros(n, np.int64), np.zeros(n, np.uint8), np.full(n, np.inf), np.zeros(n, np.uint8), (gx, gy))
    if idx.size == 0:
        return out
    with torch.no_grad():
        p = splat_params(*(_to64(a[idx]) for a in scene.arrays()), cam)
    a, b, c, det = (p[k].numpy() for k in ("a", "b", "c", "det"))
    fcl = p["frustum_clamp"].numpy()
    u, v = p["u"].numpy(), p["v"].numpy()

    mid = 0.5 * (a + c)
    lam1 = mid + np.sqrt(np.maximum(0.1, mid * mid - det))
    rr = 3.0 * np.sqrt(lam1)
    radius = np.ceil(rr)
    x_lo = np.clip(np.floor((u - radius) / tile), 0, gx)
    x_hi = np.clip(np.floor((u + radius + tile - 1) / tile), 0, gx)
    y_lo = np.clip(np.floor((v - radius) / tile), 0, gy)
    y_hi = np.clip(np.floor((v + radius + tile - 1) / tile), 0, gy)
    tiles = (x_hi - x_lo) * (y_hi - y_lo)
    ok = (det > 0) & (tiles > 0)

    # Distance (px) of each integer decision to its flip point.
    def frac_dist(val):
        return np.abs(val - np.round(val))
    gm = np.minimum.reduce([
        frac_dist(rr),
        tile * frac_dist((u - radius) / tile), tile * frac_dist((u + radius + tile - 1) / tile),
        tile * frac_dist((v - radius) / tile), tile * frac_dist((v + radius + tile - 1) / tile),
    ])

    vis = idx[ok]
    out.visible[vis] = True
    out.mean2d[vis] = np.stack([u, v], 1)[ok]
    out.conic[vis] = np.stack([p["A"].numpy(), p["B"].numpy(), p["C"].numpy()], 1)[ok]
    out.opacity[vis] = p["o"].numpy()[ok]
    out.rgb[vis] = p["rgb"].numpy()[ok]
    out.cov2d[vis] = np.stack([a, b, c], 1)[ok]
    out.radius[vis] = radius[ok].astype(np.int64)
    out.rect[vis] = np.stack([x_lo, x_hi, y_lo, y_hi], 1)[ok].astype(np.int64)
    out.tiles_touched[vis] = tiles[ok].astype(np.int64)
    raw = p["rgb_raw"].numpy()[ok]
    out.clamp_mask[vis] = ((raw[:, 0] < 0) * 1 + (raw[:, 1] < 0) * 2 + (raw[:, 2] < 0) * 4).astype(np.uint8)
    # Margins of every Gaussian in front of the camera, listed or not: an empty rectangle
    # (off-screen splat) is a decision too.
    out.geom_margin[idx] = np.where(det > 0, gm, np.inf)
    out.frustum_clamp[vis] = fcl[ok]
    return out


def params_backward(scene, cam, proj: Projected, acc9: np.ndarray):
    """Gradients of L = sum_g acc9[g] . (u, v, A, B, C, o, r, g, b)_g w.r.t. the raw parameters.

    acc9 [n,9] holds dL/d(mean2d, conic, opacity, rgb) per Gaussian. Culled
    Gaussians get exact zeros. Returns float64 arrays shaped like the inputs.
    """
    grads = [np.zeros(a.shape, np.float64) for a in scene.arrays()]
    vis = np.nonzero(proj.visible)[0]
    if vis.size == 0:
        return grads
    leaves = [_to64(a[vis]).requires_grad_(True) for a in scene.arrays()]
    p = splat_params(*leaves, cam)
    outs = torch.stack([p["u"], p["v"], p["A"], p["B"], p["C"], p["o"],
                        p["rgb"][:, 0], p["rgb"][:, 1], p["rgb"][:, 2]], dim=1)
    w = torch.tensor(np.asarray(acc9, np.float64)[vis], dtype=DT)
    g = torch.autograd.grad((outs * w).sum(), leaves, allow_unused=True)
    for k in range(5):
        if g[k] is not None:
            grads[k][vis] = g[k].numpy()
    return grads
