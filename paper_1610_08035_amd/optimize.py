"""Hyperparameter fitting: maximise the log marginal likelihood over kernel and noise
hyperparameters (the paper fits its models by scaled conjugate gradients, Sec. 4.3).

Each evaluation of logML and its gradient is one ``spingp_logml_grad`` call on a handle whose
hyperparameter buffer is updated in place (no re-assembly); the optimiser is host logic on a
few numbers per series.  The search runs over x = log(hyperparameters), which keeps every
hyperparameter positive; d(-logML)/dx = -theta * d logML/d theta.

Two optimisers: ``scg``, the scaled conjugate gradient method of Moller (Neural Networks 6,
1993), written here from its published description, and torch's L-BFGS with a strong-Wolfe
line search driving the autograd function of ``autograd.py``.
"""
from __future__ import annotations

import contextlib
from dataclasses import dataclass, field

import numpy as np
import torch

from .spingp import Handle


@dataclass
class ScgInfo:
    n_iter: int = 0
    n_eval: int = 0
    converged: bool = False
    reason: str = ""
    history: list = field(default_factory=list)   # objective after every accepted step


def scg(fun, x0, max_iter=500, gtol=1e-8, ftol=0.0, sigma0=1e-4, lambda0=1e-6):
    """Minimise fun(x) -> (value, gradient) by scaled conjugate gradients.

    Per iteration: a finite difference of gradients along the search direction p gives the
    curvature p^T H p; a Levenberg-Marquardt scale lambda keeps that curvature positive and is
    raised or lowered by the comparison parameter Delta (actual over predicted decrease).  The
    direction restarts at the negative gradient every n accepted steps (n = dimension);
    otherwise it is updated Polak-Ribiere style.  When the predicted decrease is below the
    rounding of f, the actual decrease in Delta is taken from the gradients at both ends of
    the step (trapezoid rule) instead of from the difference of two values.  Stops when
    max |gradient| <= gtol, when an accepted step lowers the objective by at most
    ftol * (1 + |f|), or after max_iter iterations.
    """
    x = np.array(x0, dtype=np.float64).reshape(-1)
    n = x.size
    f, g = fun(x)
    g = np.asarray(g, dtype=np.float64).reshape(-1)
    info = ScgInfo(n_eval=1, history=[float(f)])
    if not np.isfinite(f) or not np.all(np.isfinite(g)):
        info.reason = "non-finite objective at the start"
        return x, f, g, info
    r = -g
    p = r.copy()
    lam, lam_bar = lambda0, 0.0
    success = True
    delta = 0.0
    since_restart = 0
    for k in range(1, max_iter + 1):
        info.n_iter = k
        if np.max(np.abs(g)) <= gtol:
            info.converged, info.reason = True, "gradient"
            break
        pp = float(p @ p)
        if success:
            # curvature along p from a gradient difference over a step of length sigma0
            sig = sigma0 / np.sqrt(pp)
            _, gs = fun(x + sig * p)
            info.n_eval += 1
            s = (np.asarray(gs, dtype=np.float64).reshape(-1) - g) / sig
            delta = float(p @ s)
        # regularise the curvature with the current scale; make it positive if it is not
        delta += (lam - lam_bar) * pp
        if delta <= 0.0:
            lam_bar = 2.0 * (lam - delta / pp)
            delta = -delta + lam * pp
            lam = lam_bar
        mu = float(p @ r)
        if mu <= 0.0:
            # not a descent direction (lost conjugacy): restart from the gradient
            p = r.copy()
            success, lam_bar, since_restart = True, 0.0, 0
            continue
        alpha = mu / delta
        x_new = x + alpha * p
        f_new, g_new = fun(x_new)
        info.n_eval += 1
        g_new = np.asarray(g_new, dtype=np.float64).reshape(-1)
        ok = np.isfinite(f_new) and np.all(np.isfinite(g_new))
        Delta = 2.0 * delta * (f - f_new) / (mu * mu) if ok else -np.inf
        if ok and mu * mu / (2.0 * delta) <= 64.0 * np.finfo(np.float64).eps * max(1.0, abs(f)):
            # the predicted decrease is below the rounding of f: measure the actual decrease by
            # the trapezoid rule on the gradients along the step (exact for a quadratic)
            Delta = 2.0 * delta * (-0.5 * alpha * float(p @ (g + g_new))) / (mu * mu)
        if Delta >= 0.0:
            r_old = r
            f_old = f
            x, f, g = x_new, f_new, g_new
            r = -g
            lam_bar, success = 0.0, True
            info.history.append(float(f))
            since_restart += 1
            if since_restart >= n:
                p = r.copy()
                since_restart = 0
            else:
                beta = float(r @ r - r @ r_old) / mu
                p = r + beta * p
            if Delta >= 0.75:
                lam *= 0.25
            if ftol > 0.0 and abs(f_old - f) <= ftol * (1.0 + abs(f)):
                info.converged, info.reason = True, "objective change"
                break
        else:
            lam_bar, success = lam, False
        if Delta < 0.25:
            lam += delta * (1.0 - Delta) / pp
        if not np.isfinite(lam) or lam > 1e100:
            info.reason = "scale diverged"
            break
    else:
        info.reason = "max_iter"
    if not info.converged and not info.reason:
        info.reason = "max_iter"
    return x, f, g, info


@dataclass
class FitResult:
    hyper: np.ndarray          # [S, n_hyper] fitted hyperparameters
    logml: np.ndarray          # [S] log marginal likelihood at the fit
    grad: np.ndarray           # [S, n_hyper] d logML / d hyper at the fit
    n_iter: int
    n_eval: int
    converged: bool
    reason: str
    history: list


def fit(t, y, terms, hyper0, offsets=None, method="scg", max_iter=500, gtol=1e-7, ftol=0.0,
        fixed=None, handle=None):
    """Maximise the summed log marginal likelihood of one series or a batch over the
    hyperparameters, starting at hyper0 ([S, n_hyper] or flat, positive).

    t, y (and offsets for several series) are device tensors as for ``Handle.assemble``.
    ``fixed``: indices into a hyperparameter row held at their starting values.  Convergence:
    max |d(-logML)/d log theta| <= gtol * n_points.  ``handle``: an existing handle large
    enough for the problem (reused, re-assembled); otherwise one is created and closed.
    """
    dev = t.device
    S = 1 if offsets is None else offsets.numel() - 1
    own = handle is None
    h = Handle(terms, t.numel(), S) if own else handle
    # hyperparameter uploads and result reads are ordered with the handle's launches by running
    # them on the handle's stream
    stream = getattr(h, "stream", None)
    with torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext():
        try:
            return _fit(h, t, y, terms, hyper0, offsets, S, method, max_iter, gtol, ftol, fixed, dev)
        finally:
            if own:
                h.close()


def _fit(h, t, y, terms, hyper0, offsets, S, method, max_iter, gtol, ftol, fixed, dev):
    nh = h.n_hyper
    x0 = np.log(np.asarray(hyper0, dtype=np.float64).reshape(S, nh))
    mask = np.ones((S, nh), dtype=bool)
    if fixed is not None:
        mask[:, list(fixed)] = False
    hyp_dev = torch.tensor(np.exp(x0).reshape(-1), dtype=torch.float64, device=dev)
    h.assemble(t, y, hyp_dev, offsets if S > 1 else None)
    rc, bad = h.status()
    if rc != 0:
        raise ValueError(f"invalid inputs: status {rc} at {bad}")
    n_pts = t.numel()
    xfix = x0.copy()

    def full(xv):
        xf = xfix.copy()
        xf[mask] = xv
        return xf

    def evaluate(xf):
        hyp_dev.copy_(torch.from_numpy(np.exp(xf).reshape(-1)))
        ll, g = h.logml_grad()
        return ll.cpu().numpy(), g.cpu().numpy().reshape(S, nh)

    if method == "scg":
        def fun(xv):
            xf = full(xv)
            ll, g = evaluate(xf)
            return -float(ll.sum()), -(g * np.exp(xf))[mask]

        xv, _, _, info = scg(fun, x0[mask], max_iter=max_iter, gtol=gtol * n_pts, ftol=ftol)
        xf = full(xv)
        n_iter, n_eval, conv, reason, hist = info.n_iter, info.n_eval, info.converged, info.reason, info.history
    elif method == "lbfgs":
        from .autograd import logml as logml_fn
        xt = torch.tensor(x0, dtype=torch.float64, device=dev, requires_grad=True)
        mt = torch.tensor(mask, device=dev)
        xf0 = torch.tensor(x0, dtype=torch.float64, device=dev)
        opt = torch.optim.LBFGS([xt], lr=1.0, max_iter=max_iter, max_eval=4 * max_iter,
                                tolerance_grad=gtol * n_pts, tolerance_change=max(ftol, 1e-300),
                                history_size=20, line_search_fn="strong_wolfe")
        count = {"eval": 0}
        hist = []

        def closure():
            opt.zero_grad()
            xe = torch.where(mt, xt, xf0)
            loss = -logml_fn(t, y, xe.exp(), terms, offsets if S > 1 else None).sum()
            loss.backward()
            count["eval"] += 1
            hist.append(float(loss.item()))
            return loss

        opt.step(closure)
        xf = torch.where(mt, xt, xf0).detach().cpu().numpy()
        st = opt.state[opt._params[0]]
        n_iter, n_eval = int(st.get("n_iter", 0)), count["eval"]
        gmax = float(xt.grad.abs().max()) if xt.grad is not None else np.inf
        conv = gmax <= gtol * n_pts
        reason = "gradient" if conv else "stopped"
    else:
        raise ValueError(f"unknown method {method!r}")
    ll, g = evaluate(xf)
    return FitResult(hyper=np.exp(xf), logml=ll, grad=g, n_iter=n_iter, n_eval=n_eval,
                     converged=bool(conv), reason=reason, history=hist)
