"""torch.autograd.Function over the library's log marginal likelihood and its adjoint gradient.

`LogML.apply(t, y, hyper, terms)` returns logML per series; backward multiplies the
hyperparameter gradient of `spingp_logml_grad` (the hand-written reverse sweep, Sec. 2.4)
by the incoming gradient.  t and y are data, so they receive no gradient.
"""
from __future__ import annotations

import torch

from .spingp import Handle

_handles = {}


def _handle(terms, n, device):
    key = (tuple(tuple(x) for x in terms), device.index)
    h = _handles.get(key)
    if h is None or h.max_points < n:
        h = Handle(terms, max(n, 1024))
        h.max_points = max(n, 1024)
        _handles[key] = h
    return h


class LogML(torch.autograd.Function):
    @staticmethod
    def forward(ctx, t, y, hyper, terms):
        h = _handle(terms, t.numel(), t.device)
        hyper_c = hyper.detach().contiguous().reshape(-1)
        h.assemble(t.contiguous(), y.contiguous(), hyper_c)
        ll, g = h.logml_grad()
        ctx.save_for_backward(g)
        ctx.hshape = hyper.shape
        return ll

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        gh = (grad_out.reshape(-1, 1) * g).reshape(ctx.hshape)
        return None, None, gh, None


def logml(t, y, hyper, terms):
    return LogML.apply(t, y, hyper, terms)
