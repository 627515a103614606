"""torch.autograd.Function wrappers of the gs3 C ABI (argument marshalling only).

One Stage-1 iteration (Sec. 4.1) as an autograd graph:

    dmu, dq = NTCQuery.apply(ntc.anchor, ctx, means, token)   # Eq. 5
    image   = Render.apply(dmu, dq, ctx, gaussians, camera, slot)  # Eq. 1-4
    loss    = Loss.apply(image, target, ctx, lam)            # Eq. 6
    loss.backward()                                           # adjoints
    ctx.ntc_step(...)                                         # Adam

Every forward and backward is one call of libgs3.so; no arithmetic happens
in torch.  The NTC parameters live in the context, not in torch tensors, so
NTCQuery takes an `anchor`: a zero-size tensor that requires grad and only
gives autograd an edge into the NTC.  Its backward adds the NTC parameter
gradient into the context's gradient buffers (gs3_ntc_backward) and returns
an empty gradient for the anchor.
"""
from __future__ import annotations

import torch

from . import gs3


def ntc_anchor(device=None) -> torch.Tensor:
    """The anchor NTCQuery hangs off (zero elements, requires grad)."""
    return torch.zeros(0, device=device or "cuda", requires_grad=True)


class NTCQuery(torch.autograd.Function):
    """(dmu, dq) = NTC(means) (gs3_ntc_forward); backward: gs3_ntc_backward.
    `token` is the preparation token of the frozen means (0: none)."""

    @staticmethod
    def forward(fctx, anchor, ctx: gs3.Context, means, token: int = 0):
        dmu, dq = ctx.ntc_forward(means, token=token)
        fctx.ctx, fctx.means, fctx.token = ctx, means, token
        return dmu, dq

    @staticmethod
    def backward(fctx, g_dmu, g_dq):
        ctx, n = fctx.ctx, fctx.means.shape[0]
        g_dmu = ctx.zeros(n, 3) if g_dmu is None else g_dmu.contiguous()
        g_dq = ctx.zeros(n, 4) if g_dq is None else g_dq.contiguous()
        ctx.ntc_backward(fctx.means, g_dmu, g_dq, fctx.token)
        return torch.zeros(0, device=g_dmu.device), None, None, None


class Render(torch.autograd.Function):
    """image (3 x H x W) of the Gaussians transformed by (dmu, dq)
    (gs3_render on `slot`); backward: gs3_render_backward -> (d dmu, d dq).
    The slot keeps the render state until its backward."""

    @staticmethod
    def forward(fctx, dmu, dq, ctx: gs3.Context, gaussians: gs3.GaussiansGPU, camera, slot: int = 0):
        dmu, dq = dmu.detach().contiguous(), dq.detach().contiguous()
        image = ctx.render(gaussians, camera, dmu, dq, slot=slot)
        fctx.ctx, fctx.slot, fctx.n = ctx, slot, gaussians.n
        return image

    @staticmethod
    def backward(fctx, g_image):
        ctx, n = fctx.ctx, fctx.n
        d_dmu, d_dq = ctx.zeros(n, 3), ctx.zeros(n, 4)
        ctx.render_backward(g_image.contiguous(), {"d_dmu": d_dmu, "d_dq": d_dq}, slot=fctx.slot)
        return d_dmu, d_dq, None, None, None, None


class Loss(torch.autograd.Function):
    """Eq. 6 loss (gs3_loss), a 0-dim tensor.  gs3_loss writes dL/dimage in
    the forward; the backward hands it on.  The loss must be the root of the
    backward pass (incoming gradient 1): scaling it would be arithmetic
    outside the library."""

    @staticmethod
    def forward(fctx, image, target, ctx: gs3.Context, lam: float = 0.2):
        loss, d_image = ctx.loss(image.detach().contiguous(), target.contiguous(), lam)
        fctx.save_for_backward(d_image)
        return loss.reshape(())

    @staticmethod
    def backward(fctx, g):
        (d_image,) = fctx.saved_tensors
        if float(g) != 1.0:
            raise ValueError("Loss must be the root of the backward pass (incoming gradient 1)")
        return d_image, None, None, None
