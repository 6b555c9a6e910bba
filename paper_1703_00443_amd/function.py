"""torch.autograd.Function over the batched QP solver (Section 3, the OptNet layer).

    z = qp_layer(Q, q, A, b, G, h, opts=None)

Forward runs qp_forward_batched; backward runs qp_backward_batched with the
factor the forward stored (Section 3.1.1: no new factorization).  Any of Q, q,
A, b, G, h may omit the batch dimension (shared by the whole batch); their
gradients are then summed over the batch.  A/b and G/h may be None.
Argument marshalling only: all arithmetic runs in libqpmi.so.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import binding

_NDIM = {"Q": 3, "q": 2, "A": 3, "b": 2, "G": 3, "h": 2}


class QPFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, Q, q, A, b, G, h, opts: Optional[binding.qp_opts] = None):
        prob = binding.make_problem(Q.detach(), q.detach(),
                                    None if A is None else A.detach(),
                                    None if b is None else b.detach(),
                                    None if G is None else G.detach(),
                                    None if h is None else h.detach())
        o = opts if opts is not None else binding.default_opts(Q.dtype)
        fw = binding.forward(prob, o)
        ctx.prob, ctx.fw, ctx.opts = prob, fw, o
        ctx.shapes = {k: (None if t is None else t.shape)
                      for k, t in zip("Q q A b G h".split(), (Q, q, A, b, G, h))}
        # the layer differentiates z only (Section 3: Jacobians of lambda, nu not considered)
        ctx.mark_non_differentiable(fw.lam, fw.nu, fw.status, fw.iters)
        return fw.z, fw.lam, fw.nu, fw.status, fw.iters

    @staticmethod
    def backward(ctx, dz, dlam, dnu, dstatus, diters):
        names = "Q q A b G h".split()
        need = tuple(n for n, ng in zip(names, ctx.needs_input_grad[:6]) if ng)
        if dz is None or not need:
            return (None,) * 7
        g = binding.backward(ctx.prob, ctx.fw, dz, ctx.opts, need=need)
        outs = []
        for name in names:
            shape = ctx.shapes[name]
            t = getattr(g, "d" + name)
            if shape is None or t is None or name not in need:
                outs.append(None)
                continue
            if len(shape) < _NDIM[name]:
                t = t.sum(0)
            elif shape[0] == 1 and t.shape[0] != 1:
                t = t.sum(0, keepdim=True)
            outs.append(t.reshape(shape))
        return tuple(outs) + (None,)


def qp_layer(Q, q, A=None, b=None, G=None, h=None, opts=None, full=False):
    """Solve the batch and return z (or (z, lam, nu, status, iters) with full=True)."""
    out = QPFunction.apply(Q, q, A, b, G, h, opts)
    return out if full else out[0]
