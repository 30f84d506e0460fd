"""torch.autograd.Function over the HIP path: forward = LoD select + render,
backward = recompute-based blend backward + projection/SH backward.

The differentiable inputs are the scene's own parameter tensors (layout
order): gradients reach every node that the cut selected, interior merged
nodes included (the paper updates only the cut set's parameters, init and
training appendix).  Two gradient modes:

* default: dense gradients shaped like the parameters (torch semantics);
* ``accumulate_into=dict``: the backward adds into the given node-indexed
  arrays (e.g. pre-allocated ``.grad`` buffers) and returns no gradient,
  which avoids a dense zero-fill and add per view on large scenes.

One frame serves one view in flight: run the backward of a render before
the next render on the same frame (use one frame per view of a batch).
"""
from __future__ import annotations

import torch

from .lodgs import Frame, grads_like

PARAM_NAMES = ("means", "log_scales", "quats", "opacity_logits", "sh")


class LodSplat(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity_logits, sh, frame: Frame, cam, tau: float, bg,
                cull: bool, accumulate_into):
        scene = frame.scene
        for name, t in zip(PARAM_NAMES, (means, log_scales, quats, opacity_logits, sh)):
            if t.data_ptr() != scene.params[name].data_ptr():
                raise ValueError(f"{name} must be the scene's own parameter tensor")
        frame.lod_select(cam, tau, cull=cull)
        img = frame.render(cam, bg=bg)
        ctx.frame = frame
        ctx.accumulate_into = accumulate_into
        return img

    @staticmethod
    def backward(ctx, grad_img):
        frame = ctx.frame
        g = grad_img.contiguous()
        if g.dtype != torch.float32:
            g = g.float()
        if ctx.accumulate_into is not None:
            frame.backward(g, nodes=ctx.accumulate_into)
            return (None,) * 11
        grads = grads_like(frame.scene)
        frame.backward(g, nodes=grads)
        return tuple(grads[k] for k in PARAM_NAMES) + (None,) * 6


def render_lod(frame: Frame, cam, tau: float, bg=(0.0, 0.0, 0.0), cull: bool = True, accumulate_into=None):
    """Differentiable LoD render of one view; returns the image [H, W, 3]."""
    P = frame.scene.params
    return LodSplat.apply(P["means"], P["log_scales"], P["quats"], P["opacity_logits"], P["sh"], frame, cam,
                          float(tau), tuple(float(x) for x in bg), bool(cull), accumulate_into)
