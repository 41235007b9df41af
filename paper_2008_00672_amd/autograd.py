"""torch.autograd binding of the FC synthesis (complex64 I/O).

``fc_tx(plan, x, w)`` returns tx(x) with the plan's weights set to ``w``
(all subbands' weights concatenated in plan order, fftshifted within a
subband, float32 on the plan's device). Backward runs the library's kernels:
grad_x = adjoint(grad_y) (the synthesis is complex-linear in x, so its
adjoint is the vector-Jacobian product), grad_w[p] = Re <grad_y, b_p> with
b_p the output for a unit weight at bin p (fc_tx_weight_grad). PyTorch's
conjugate-Wirtinger convention is used throughout.
"""
import torch

from .fc import OP_TX


def _set_all(plan, w):
    plan.set_all_weights(w)


class FcTx(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, w, plan):
        if plan.io != "c64":
            raise ValueError("autograd needs a complex64 (FC_IO_C64) plan")
        total = sum(s["n_short"] for s in plan.subbands)
        if w.dtype != torch.float32 or w.numel() != total:
            raise ValueError("w must hold %d float32 weights" % total)
        w = w.detach().contiguous()
        x = x.detach().contiguous()
        _set_all(plan, w)
        y = plan.tx(x)
        ctx.plan = plan
        ctx.save_for_backward(x, w)
        return y

    @staticmethod
    def backward(ctx, gy):
        x, w = ctx.saved_tensors
        plan = ctx.plan
        gy = gy.contiguous()
        # another forward may have changed the plan's weights since
        _set_all(plan, w)
        gx = plan.adjoint(gy) if ctx.needs_input_grad[0] else None
        gw = plan.weight_grad(x, gy) if ctx.needs_input_grad[1] else None
        return gx, gw, None


def fc_tx(plan, x, w):
    """Differentiable FC synthesis: y = tx(x; w)."""
    lo, _ = plan.layout(OP_TX)
    if x.numel() != int(lo[-1]):
        raise ValueError("x must hold %d low-rate samples" % int(lo[-1]))
    return FcTx.apply(x, w, plan)
