"""fp64 oracle: image losses and dL/dimage.

TEST INFRASTRUCTURE ONLY. The paper only says the loss is the difference of
the rendered and reference RGB values (Background, differentiable-rendering
training pipeline); the forms below are the 3D Gaussian Splatting ones:

  L1      = mean |I - target| over 3HW values; dL/dI = sign(I - target) / (3HW), sign(0) = 0
  D-SSIM  = 1 - SSIM, SSIM with an 11x11 Gaussian window (sigma 1.5, normalised),
            zero-padded same-size convolution per channel, C1 = 0.01^2, C2 = 0.03^2,
            averaged over 3HW
  mixed   = (1 - 0.2) L1 + 0.2 D-SSIM

Gradients come from torch.autograd in float64.
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F


def gaussian_window(size=11, sigma=1.5):
    """[size,size] float64 window: outer product of the sampled 1-D Gaussian, normalised to sum 1."""
    x = torch.arange(size, dtype=torch.float64) - (size - 1) / 2.0
    g = torch.exp(-(x * x) / (2 * sigma * sigma))
    g = g / g.sum()
    return torch.outer(g, g)


def ssim_map(img: torch.Tensor, ref: torch.Tensor) -> torch.Tensor:
    """Per-pixel SSIM [3,H,W] of two [3,H,W] float64 images (window statistics with zero padding)."""
    w = gaussian_window().expand(3, 1, 11, 11).contiguous()
    x, y = img[None], ref[None]
    mu_x = F.conv2d(x, w, padding=5, groups=3)
    mu_y = F.conv2d(y, w, padding=5, groups=3)
    sxx = F.conv2d(x * x, w, padding=5, groups=3) - mu_x * mu_x
    syy = F.conv2d(y * y, w, padding=5, groups=3) - mu_y * mu_y
    sxy = F.conv2d(x * y, w, padding=5, groups=3) - mu_x * mu_y
    c1, c2 = 0.01 ** 2, 0.03 ** 2
    s = ((2 * mu_x * mu_y + c1) * (2 * sxy + c2)) / ((mu_x * mu_x + mu_y * mu_y + c1) * (sxx + syy + c2))
    return s[0]


def ssim(img: torch.Tensor, ref: torch.Tensor) -> torch.Tensor:
    """Mean SSIM of two [3,H,W] float64 images (the mean of ssim_map over 3HW values)."""
    return ssim_map(img, ref).mean()


def loss_and_grad(image: np.ndarray, target: np.ndarray, kind: str = "l1", lam: float = 0.2):
    """Returns (loss, dL/dimage) for image/target [3,H,W]; dL/dimage is float64."""
    img = torch.tensor(np.asarray(image, np.float64), requires_grad=True)
    ref = torch.tensor(np.asarray(target, np.float64))
    l1 = (img - ref).abs().mean()
    if kind == "l1":
        loss = l1
    elif kind == "l1_dssim":
        loss = (1 - lam) * l1 + lam * (1 - ssim(img, ref))
    else:
        raise ValueError(kind)
    (g,) = torch.autograd.grad(loss, img)
    return float(loss.detach()), g.numpy()
