"""fp64 CPU oracle for the 3D Gaussian Splatting render and backward pass.

TEST INFRASTRUCTURE ONLY. Only tests/, the smoke check in __graft_entry__.py
and the CPU baseline leg of bench.py may import, call, link or execute
anything in this package. The product path (the HIP library and its Python
binding) never does, and shares no code with it.

  preprocess.py  per-Gaussian projection, EWA covariance, colour; chain rule
                 back to raw parameters by float64 autograd
  composite.py   tile lists (numpy lexsort) and the per-pixel C loops
  raster.c       front-to-back compositing and its exact derivative, in double
  loss.py        L1 and D-SSIM losses and dL/dimage

Parity pins: tests/test_oracle_*.py (closed forms, invariants, brute force
and central finite differences).
"""
from .preprocess import (project, params_backward, splat_params, sh_basis, quat_to_rot, depth_key_f32,
                         sh_constants, covariance3d)
from .composite import render, backward, composite_backward, tile_lists, pixel_entries, build_raster_lib
from .loss import loss_and_grad, ssim, ssim_map, gaussian_window
from .adam import adam_step

__all__ = [
    "project", "params_backward", "splat_params", "sh_basis", "quat_to_rot", "depth_key_f32", "sh_constants", "covariance3d",
    "render", "backward", "composite_backward", "tile_lists", "pixel_entries", "build_raster_lib",
    "loss_and_grad", "ssim", "ssim_map", "gaussian_window", "adam_step",
]
