"""torch.autograd.Function over the gsr render and backward.

The forward runs gsr_render (projection, binning, forward composite) and
keeps the library's forward state, which holds the per-pixel final
transmittance and last-contributor position so the backward recomputes each
pixel's walk instead of storing per-sample alphas. The backward runs
gsr_backward (backward composite with the configured reduction mode, then the
per-Gaussian chain rule) and returns dL/d(means3d, log_scales, quats,
opacity_logits, sh). The state borrows the parameter tensors; it is kept with
them until the backward runs or the graph is freed.
"""
from __future__ import annotations

import weakref

import torch

from . import gsr


class _State:
    """Owns one library forward state; released exactly once."""

    def __init__(self, renderer: gsr.Renderer, frame: gsr.Frame):
        self.renderer = renderer
        self.frame = frame
        self._finalizer = weakref.finalize(self, _State._release, renderer, frame)

    @staticmethod
    def _release(renderer, frame):
        if frame.state and renderer.ctx:
            renderer.release(frame)

    def release(self):
        self._finalizer()


class GaussianRasterize(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means3d, log_scales, quats, opacity_logits, sh, renderer, camera, config, sh_degree):
        tensors = [t.contiguous() for t in (means3d, log_scales, quats, opacity_logits, sh)]
        for t in tensors:
            if t.dtype != torch.float32 or not t.is_cuda:
                raise ValueError("GaussianRasterize takes fp32 CUDA tensors")
        scene = gsr.make_scene(*tensors, sh_degree)
        frame = renderer.render(scene, camera, config)
        ctx.state = _State(renderer, frame)
        ctx.config = config
        ctx.save_for_backward(*tensors)   # the forward state borrows these
        return frame.image

    @staticmethod
    def backward(ctx, grad_image):
        tensors = ctx.saved_tensors
        grads = [torch.zeros_like(t) for t in tensors]
        st = ctx.state
        st.renderer.backward(st.frame, grad_image.contiguous(), gsr.make_grads(*grads), 0, ctx.config)
        st.release()
        return (*grads, None, None, None, None)


def rasterize(means3d, log_scales, quats, opacity_logits, sh, renderer: gsr.Renderer, camera: gsr.gsr_camera,
              config: gsr.gsr_config | None = None, sh_degree: int | None = None):
    """Differentiable render: returns the [3,H,W] image; backward gives the five parameter gradients."""
    if config is None:
        config = gsr.make_config(16, 256, gsr.GSR_BWD_WAVE_REDUCE, 4, gsr.GSR_FLAG_LANE_SPLIT_ATOMICS)
    if sh_degree is None:
        k = sh.shape[1]
        sh_degree = {1: 0, 4: 1, 9: 2, 16: 3}[k]
    return GaussianRasterize.apply(means3d, log_scales, quats, opacity_logits, sh, renderer, camera, config,
                                   sh_degree)
