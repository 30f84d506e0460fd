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

Views of a batch may run on several streams (call render_lod under
``torch.cuda.stream(s)``; autograd runs each view's backward on its
forward's stream).  With ``scatter_stream`` (accumulate_into mode) the
frame-local half of a view's backward (blend backward and per-splat sums)
runs there, and the half that adds into the shared node arrays runs on
scatter_stream, in the order the autograd engine calls the backwards, so
views on different streams never update the arrays at once and the sums
are those of one stream.  The caller waits for scatter_stream before it
reads the arrays; a frame's next forward waits for its last scatter.

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
                cull: bool, accumulate_into, scatter_stream):
        scene = frame.scene
        for name, t in zip(PARAM_NAMES, (means, log_scales, quats, opacity_logits, sh)):
            if t.data_ptr() != scene.params[name].data_ptr():
                raise ValueError(f"{name} must be the scene's own parameter tensor")
        if scatter_stream is not None and accumulate_into is None:
            raise ValueError("scatter_stream needs accumulate_into")
        done = getattr(frame, "_scatter_done", None)
        if done is not None:  # the frame's last scatter still reads its state
            torch.cuda.current_stream().wait_event(done)
        frame.lod_select(cam, tau, cull=cull)
        img = frame.render(cam, bg=bg)
        ctx.frame = frame
        ctx.accumulate_into = accumulate_into
        ctx.scatter_stream = scatter_stream
        return img

    @staticmethod
    def backward(ctx, grad_img):
        frame = ctx.frame
        g = grad_img.contiguous()
        if g.dtype != torch.float32:
            g = g.float()
        none = (None,) * 12
        if ctx.scatter_stream is not None:
            cur = torch.cuda.current_stream()
            frame.backward(g, stream=cur, phases="partials")
            ready = torch.cuda.Event()
            ready.record(cur)
            ctx.scatter_stream.wait_event(ready)
            frame.backward(None, nodes=ctx.accumulate_into, stream=ctx.scatter_stream, phases="scatter")
            done = torch.cuda.Event()
            done.record(ctx.scatter_stream)
            frame._scatter_done = done
            return none
        if ctx.accumulate_into is not None:
            frame.backward(g, nodes=ctx.accumulate_into)
            return none
        grads = grads_like(frame.scene)
        frame.backward(g, nodes=grads)
        return tuple(grads[k] for k in PARAM_NAMES) + (None,) * 7


def render_lod(frame: Frame, cam, tau: float, bg=(0.0, 0.0, 0.0), cull: bool = True, accumulate_into=None,
               scatter_stream=None):
    """Differentiable LoD render of one view; returns the image [H, W, 3]."""
    P = frame.scene.params
    return LodSplat.apply(P["means"], P["log_scales"], P["quats"], P["opacity_logits"], P["sh"], frame, cam,
                          float(tau), tuple(float(x) for x in bg), bool(cull), accumulate_into, scatter_stream)
