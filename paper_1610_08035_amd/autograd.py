"""torch.autograd.Function over the library's log marginal likelihood and its adjoint gradient.

`LogML.apply(t, y, hyper, terms, offsets=None)` returns logML per series (hyper: [S, n_hyper] or
flat); backward multiplies the hyperparameter gradient of `spingp_logml_grad` (the hand-written
reverse sweep, Sec. 2.4) by the incoming gradient.  t and y are data and get no gradient.  One
handle per (model, device, size class) is kept and reused, so repeated calls allocate nothing
in the library.
"""
from __future__ import annotations

import torch

from .spingp import Handle

_handles = {}


def _handle(terms, n, s, device):
    key = (tuple(tuple(x) for x in terms), device.index, s > 1)
    h = _handles.get(key)
    if h is None or h.max_points < n or h.max_series < s:
        if h is not None:
            h.close()
        mp = max(n, 1024 if h is None else 2 * h.max_points)
        ms = max(s, 1 if h is None else h.max_series)
        h = Handle(terms, mp, ms)
        h.max_points, h.max_series = mp, ms
        _handles[key] = h
    return h


class LogML(torch.autograd.Function):
    @staticmethod
    def forward(ctx, t, y, hyper, terms, offsets=None):
        s = 1 if offsets is None else offsets.numel() - 1
        h = _handle(terms, t.numel(), s, t.device)
        hyper_c = hyper.detach().contiguous().reshape(-1)
        h.assemble(t.contiguous(), y.contiguous(), hyper_c, offsets if s > 1 else None)
        ll, g = h.logml_grad()
        ctx.save_for_backward(g)
        ctx.hshape = hyper.shape
        return ll

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        gh = (grad_out.reshape(-1, 1) * g).reshape(ctx.hshape)
        return None, None, gh, None, None


def logml(t, y, hyper, terms, offsets=None):
    return LogML.apply(t, y, hyper, terms, offsets)
