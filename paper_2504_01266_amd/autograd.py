"""torch.autograd wrapper of the filter: forward and both adjoints run in the
HIP library (filter2d_forward / filter2d_backward); torch only allocates and
passes its current stream."""
import torch

from . import binding as B


class Filter2dFn(torch.autograd.Function):
    """y = filter2d(x, f) with clamp-to-edge borders.

    SHARED / BANK return one tensor; DEPTHWISE returns one tensor per filter
    index (filter c*m+j of channel c goes to output j)."""

    @staticmethod
    def forward(ctx, image, filt, mode="shared"):
        ctx.mode = mode
        ctx.save_for_backward(image, filt)
        out = B.forward(image, filt, mode=mode)
        if isinstance(out, list):
            return tuple(out)
        return out

    @staticmethod
    def backward(ctx, *grads):
        image, filt = ctx.saved_tensors
        need_x, need_f = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if not (need_x or need_f):
            return None, None, None
        like = image if image.dim() == 4 else image.unsqueeze(0)
        gs = []
        for g in grads:
            if g is None:
                g = torch.zeros(like.shape, dtype=torch.float32, device=image.device)
            gs.append(g.contiguous())
        gi, gf = B.backward(image, filt, gs, mode=ctx.mode, need_input=need_x, need_filter=need_f)
        if gi is not None:
            gi = gi.view(image.shape).to(image.dtype)
        if gf is not None:
            gf = gf.view(filt.shape).to(filt.dtype)
        return gi, gf, None


def filter2d(image, filt, mode="shared"):
    """Differentiable K x K filter (correlation, clamp-to-edge borders)."""
    return Filter2dFn.apply(image, filt, mode)
