"""torch.autograd wrapper: forward and hand-written backward in the HIP library."""

import torch


class _LatticeSplineFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, spline, x, sched, *coeffs):
        vol = spline.bind([c.detach().contiguous() for c in coeffs])
        xd = x.detach().contiguous()
        schedule = spline.schedule(vol, xd) if sched else None
        f = spline.eval(vol, xd, schedule=schedule)
        ctx.spline, ctx.vol, ctx.schedule, ctx.xd = spline, vol, schedule, xd
        return f

    @staticmethod
    def backward(ctx, gf):
        want_x = ctx.needs_input_grad[1]
        want_c = any(ctx.needs_input_grad[3:])
        grad_c, grad_x = ctx.spline.adjoint(ctx.vol, ctx.xd, gf.contiguous().float(), grad_x=want_x,
                                            schedule=ctx.schedule)
        if not want_c:
            grad_c = [None] * len(grad_c)
        else:
            grad_c = [g.to(c.dtype) for g, c in zip(grad_c, ctx.vol.coeffs)]
        return (None, grad_x if want_x else None, None, *grad_c)


def lattice_spline(spline, x, coeffs, schedule=None):
    """f = sum_n c_n phi(x - n) with gradients for x and every coset array.
    schedule: True to sort the queries into cache-friendly order (shared by
    forward and backward); default: only for batches above 2^16 queries."""
    sched = (x.shape[0] > (1 << 16)) if schedule is None else bool(schedule)
    return _LatticeSplineFn.apply(spline, x, sched, *coeffs)
