"""Shared helpers of the GPU parity tests (comparison bars and device transfer)."""
from __future__ import annotations

import numpy as np

# Bars (FP64).  mean: |dm| <= 1e-9 (|m| + sqrt(v)); variance: |dv| <= 1e-9 v; logML: 1e-8 relative;
# gradient: 1e-7 relative per component with a floor of 1e-3 * max|g| (components that are
# nearly zero by cancellation are compared on the scale of the largest one).
TOL_MEAN = 1e-9
TOL_VAR = 1e-9
TOL_LOGML = 1e-8
TOL_GRAD = 1e-7


def to_dev(a, dtype=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype or torch.float64, device="cuda:0")


def check_logml(got, ref, tol=TOL_LOGML):
    err = abs(got - ref) / abs(ref)
    assert err <= tol, f"logML {got!r} vs {ref!r}: rel {err:.3e} > {tol:g}"


def check_mean_var(fm, fv, ref_m, ref_v):
    scale = np.abs(ref_m) + np.sqrt(np.maximum(ref_v, 0.0))
    em = np.abs(fm - ref_m) / scale
    ev = np.abs(fv - ref_v) / ref_v
    i, j = int(np.argmax(em)), int(np.argmax(ev))
    assert em[i] <= TOL_MEAN, f"mean at {i}: {fm[i]!r} vs {ref_m[i]!r} ({em[i]:.3e})"
    assert ev[j] <= TOL_VAR, f"variance at {j}: {fv[j]!r} vs {ref_v[j]!r} ({ev[j]:.3e})"


def check_grad(g, ref, tol=TOL_GRAD):
    g = np.asarray(g, dtype=np.float64).reshape(-1)
    ref = np.asarray(ref, dtype=np.float64).reshape(-1)
    scale = np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
    err = np.abs(g - ref) / scale
    assert err.max() <= tol, f"gradient {g} vs {ref}: rel {err.max():.3e} > {tol:g}"
