"""torch.autograd wrapper: forward and hand-written backward in the HIP library."""

import torch


class _LatticeSplineFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, spline, x, *coeffs):
        vol = spline.bind([c.detach().contiguous() for c in coeffs])
        f = spline.eval(vol, x.detach().contiguous())
        ctx.spline, ctx.vol = spline, vol
        ctx.save_for_backward(x)
        return f

    @staticmethod
    def backward(ctx, gf):
        (x,) = ctx.saved_tensors
        want_x = ctx.needs_input_grad[1]
        want_c = any(ctx.needs_input_grad[2:])
        grad_c, grad_x = ctx.spline.adjoint(ctx.vol, x.detach().contiguous(), gf.contiguous().float(),
                                            grad_x=want_x)
        if not want_c:
            grad_c = [None] * len(grad_c)
        else:
            grad_c = [g.to(c.dtype) for g, c in zip(grad_c, ctx.vol.coeffs)]
        return (None, grad_x if want_x else None, *grad_c)


def lattice_spline(spline, x, coeffs):
    """f = sum_n c_n phi(x - n) with gradients for x and every coset array."""
    return _LatticeSplineFn.apply(spline, x, *coeffs)
